"""Statistical parity of the full path (decay sampling, transport, tally,
Eq. 1-3) against the oracle's exact-traversal mode, which shares neither the
tracking algorithm, the Klein-Nishina sampler nor the random streams with the
device.  Bars (the stated tolerance of the method): every organ within three
combined standard errors of the organ mean, and a voxel chi-square with
p > 0.01 over voxels with density >= 0.01 g/cm^3 and relative error <= 5 % in
both runs.  The device ledger closes to 1e-9."""
import json
import os

import numpy as np
import pytest
from scipy import stats

from conftest import ledger_balance, oracle_phantom
from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu


def _gpu(engine, pid, prob, n, seed):
    engine.set_problem(pid, prob)
    engine.run(pid, n, seed, photons_per_decay=prob.photons_per_decay)
    rate, rel = engine.dose(pid)
    r_o, e3, sig = engine.organs(pid)
    return (rate.cpu().numpy(), rel.cpu().numpy(), r_o, sig, engine.ledger(pid),
            engine.stats(pid))


def _oracle(orc, prob, n, seed):
    ph = oracle_phantom(orc, prob)
    tal, _ = orc.run(ph, n, seed, photons_per_decay=prob.photons_per_decay)
    a = prob.total_activity_bq
    rate, eps = orc.finalize(ph, tal, a)
    r_o, sig = orc.organ_mean_sigma(tal, a)
    return rate, eps, r_o, sig, tal


def _organ_z(gr, gs, orr, os_):
    m = (gr > 0) & (orr > 0)
    z = (gr[m] - orr[m]) / np.sqrt((gr[m] * gs[m]) ** 2 + (orr[m] * os_[m]) ** 2)
    return z, m


def _voxel_p(gd, ge, od, oe, rho):
    m = (rho >= 0.01) & (ge > 0) & (oe > 0) & (ge <= 0.05) & (oe <= 0.05)
    chi2 = (((gd - od) ** 2)[m] / ((gd * ge) ** 2 + (od * oe) ** 2)[m]).sum()
    return stats.chi2.sf(chi2, m.sum()), m.sum(), chi2 / max(m.sum(), 1)


@pytest.mark.parametrize("name", ["water64", "slab128", "patient"])
def test_statistical_parity(engine, orc, name):
    """Live oracle runs sized to finish in seconds."""
    if name == "water64":
        prob, ng, no, nv_min = P.water_point_source(n=64, voxel_mm=2.0), 10 ** 7, 10 ** 7, 300
    elif name == "slab128":
        prob, ng, no, nv_min = P.slab_phantom(), 10 ** 7, 2 * 10 ** 6, 150
    else:  # too few voxels reach 5 % at these sizes: organs only
        # the oracle sample sets the power here: at 10^6 decays the scores of
        # the small organs (tens of histories hit them) are too skewed for the
        # normal bar, and seed 2002's Spinal_Cord mean sits 3.1 sigma from the
        # oracle's own 10^8-decay run; at 4 x 10^6 it sits within 1.8
        prob, ng, no, nv_min = P.patient_phantom(), 10 ** 7, 4 * 10 ** 6, 0
    gd, ge, gr, gs, led, st = _gpu(engine, 20, prob, ng, 1001)
    od, oe, orr, os_, _ = _oracle(orc, prob, no, 2002)
    assert abs(ledger_balance(led)) < 1e-9
    assert st["overflows"] == 0 and st["histories"] == ng
    z, m = _organ_z(gr, gs, orr, os_)
    print(name, "organ z:", np.round(z, 2))
    assert m.sum() >= min(prob.n_organs, 10)
    assert np.all(np.abs(z) <= 3.0)
    if nv_min:
        p, nv, red = _voxel_p(gd, ge, od, oe, prob.density)
        print(name, "voxel chi2/dof %.4f over %d voxels, p = %.4f" % (red, nv, p))
        assert nv >= nv_min and p > 0.01


def test_statistical_parity_photon_cutoff(engine, orc):
    """The slab with Section 2.1's photon cutoff raised to 150 keV, against
    the exact-traversal oracle with the same cutoff: organs within three
    combined sigma, the voxel chi-square, a cutoff deposit on both sides and
    both ledgers closed."""
    prob = P.slab_phantom()
    engine.set_problem(23, prob)
    engine.run(23, 10 ** 7, 3003, photon_cutoff_mev=0.15)
    gd, ge = (t.cpu().numpy() for t in engine.dose(23))
    gr, _, gs = engine.organs(23)
    led = engine.ledger(23)
    ph = oracle_phantom(orc, prob)
    # 10^7 oracle decays: at 2 x 10^6 the voxels that pass the 5 % cut are
    # chosen on a noisy sigma estimate, which inflates the chi-square (two
    # oracle runs, 10^7 and 2 x 10^6 decays, already give chi2/dof 1.2 there)
    tal, _ = orc.run(ph, 10 ** 7, 4004, cutoff_mev=0.15)
    a = prob.total_activity_bq
    od, oe = orc.finalize(ph, tal, a)
    orr, os_ = orc.organ_mean_sigma(tal, a)
    oled = tal.ledger
    assert led["dep_cutoff"] > 0.0 and oled["dep_cutoff"] > 0.0
    assert abs(ledger_balance(led)) < 1e-9 and abs(ledger_balance(oled)) < 1e-9
    # the cutoff's share of the deposited energy agrees within its binomial noise
    share = lambda l: l["dep_cutoff"] / (l["dep_compton"] + l["dep_pe"] + l["dep_cutoff"])  # noqa: E731
    assert share(led) == pytest.approx(share(oled), rel=2e-2, abs=0)
    z, m = _organ_z(gr, gs, orr, os_)
    print("cutoff 150 keV organ z:", np.round(z, 2))
    assert m.sum() >= 8 and np.all(np.abs(z) <= 3.0)
    p, nv, red = _voxel_p(gd, ge, od, oe, prob.density)
    print("cutoff 150 keV voxel chi2/dof %.4f over %d voxels, p = %.4f" % (red, nv, p))
    assert nv >= 1000 and p > 0.01


def _reference():
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_reference.json")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["slab128", "patient"])
def test_parity_at_1e8_against_stored_oracle(engine, name):
    """GPU at 10^8 decays against the oracle's stored 10^8-decay run
    (tests/golden/make_oracle_reference.py): every organ within three combined
    sigma, within 1 % wherever three combined sigma are below 1 %, and the
    voxel chi-square over the oracle's voxels with <= 5 % uncertainty."""
    ref = _reference()[name]
    prob = P.slab_phantom() if name == "slab128" else P.patient_phantom()
    gd, ge, gr, gs, led, st = _gpu(engine, 22, prob, ref["n_decays"], 6007)
    assert abs(ledger_balance(led)) < 1e-9 and st["overflows"] == 0
    orr = np.array(ref["organ_rate"])
    os_ = np.array(ref["organ_rel_sigma"])
    z, m = _organ_z(gr, gs, orr, os_)
    rel = (gr[m] - orr[m]) / orr[m]
    comb = np.sqrt((gr[m] * gs[m]) ** 2 + (orr[m] * os_[m]) ** 2) / orr[m]
    print(name, "organ z:", np.round(z, 2))
    print(name, "organ rel diff %:", np.round(100 * rel, 3))
    assert np.all(np.abs(z) <= 3.0)
    tight = 3 * comb <= 0.01
    assert tight.sum() >= (5 if name == "patient" else 3)
    assert np.all(np.abs(rel[tight]) <= 0.01)
    idx = np.array(ref["voxel_index"], dtype=np.int64)
    od, oe = np.array(ref["voxel_rate"]), np.array(ref["voxel_rel"])
    g, e = gd.ravel()[idx], ge.ravel()[idx]
    keep = (e > 0) & (e <= 0.05)
    chi2 = (((g - od) ** 2)[keep] / ((g * e) ** 2 + (od * oe) ** 2)[keep]).sum()
    p = stats.chi2.sf(chi2, keep.sum())
    print(name, "voxel chi2/dof %.4f over %d voxels, p = %.4f" % (chi2 / keep.sum(),
                                                                    keep.sum(), p))
    assert keep.sum() >= 1000 and p > 0.01


@pytest.mark.parametrize("full", [False, True])
def test_eq2_two_ways_on_device(engine, full):
    """The per-history organ scores summed over histories equal Eq. 2 applied
    to the voxel tally.  On the full-size patient about a quarter of the
    histories deposit in more voxels than the registers hold, and about one
    in a hundred in more than registers and LDS together, so every tier of
    the deposit list and the organ merge over it is exercised."""
    if full:
        prob = P.patient_phantom()
    else:
        prob = P.patient_phantom(shape=(80, 64, 64), voxel_mm=(8.0, 8.0, 12.0), seed=9)
    engine.set_problem(21, prob)
    engine.run(21, 2 * 10 ** 6, 5)
    if full:  # histories over more organs than the slots hold merge from the list
        assert engine.stats(21)["list_merges"] > 1000
    r2, _, _ = engine.organs(21)
    rs = B.nmd_get_organ_score(engine.ctx, 21, prob.n_organs)
    nz = r2 > 0
    assert nz.sum() >= 20
    assert np.allclose(rs[nz], r2[nz], rtol=1e-10, atol=0)
