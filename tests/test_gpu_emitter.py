"""Gamma + beta emitters on the device (nmd_set_emitter), with the 177Lu
and 131I data of tests/golden/*_decay.json: history by history against the
oracle's emitter on the same streams, statistically against exact traversal
on the patient, and the switch's semantics."""
import json
import os

import numpy as np
import pytest

from conftest import ledger_balance, oracle_phantom
from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu


def _nuclide(name):
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name + "_decay.json")))
    return ([e * 1e-3 for e in d["gamma_lines_kev"]], d["gamma_yields_per_decay"],
            d["beta_minus_mean_kev"] * 1e-3)


# 131I's lines reach 723 keV: its phantom takes the wide grid (1 keV to 1 MeV)
EMITTERS = {"lu177": _nuclide("lu177"), "i131": _nuclide("i131")}
LINES, YIELDS, BETA = EMITTERS["lu177"]


def _balance(led):
    return ledger_balance(led) + led["dep_beta"] / led["emitted"]


@pytest.mark.parametrize("nuclide", ["lu177", "i131"])
def test_emitter_replays_history_by_history(engine, orc, nuclide):
    """The slab's point source: the line choice, the beta deposit and the
    photon's events replay the oracle's emitter draw for draw."""
    LINES, YIELDS, BETA = EMITTERS[nuclide]
    prob = P.slab_phantom(n=64, voxel_mm=6.0)
    engine.set_problem(61, prob)
    B.nmd_set_emitter(engine.ctx, 61, LINES, YIELDS, BETA)
    n = 30_000
    t = engine.torch
    rec = t.zeros(n * 10, dtype=t.float64, device=engine.device)
    engine.run(61, n, 41, history_records=rec)
    g = rec.cpu().numpy().reshape(n, 10)
    tal, o = orc.run(oracle_phantom(orc, prob), n, 41, tracking=orc.TRACK_WOODCOCK, pid=61,
                     history_records=True, emitter=(LINES, YIELDS, BETA))
    same = np.all(g[:, [2, 3, 4, 5, 8]] == o[:, [2, 3, 4, 5, 8]], axis=1)
    assert same.mean() >= 0.995, same.mean()
    e_ok = np.abs(g[:, 0] - o[:, 0]) <= 1e-5 + 1e-5 * np.abs(o[:, 0])
    x_ok = np.abs(g[:, 1] - o[:, 1]) <= 1e-5 + 1e-5 * np.abs(o[:, 1])
    assert (same & e_ok & x_ok).mean() >= 0.995
    led = engine.ledger(61)
    assert abs(_balance(led)) < 1e-9 and abs(_balance(tal.ledger)) < 1e-9
    assert led["dep_beta"] == pytest.approx(n * BETA, rel=1e-6)
    st = engine.stats(61)
    assert st["photons"] == tal.stats["photons"]
    assert abs(st["photons"] / n - sum(YIELDS)) < 5 * np.sqrt(sum(YIELDS) / n)


@pytest.mark.parametrize("nuclide", ["lu177", "i131"])
def test_emitter_statistical_parity_patient(engine, orc, nuclide):
    """The full-size patient with the emitter against the exact-traversal
    oracle with the same emitter: every organ within three combined sigma."""
    LINES, YIELDS, BETA = EMITTERS[nuclide]
    prob = P.patient_phantom()
    engine.set_problem(62, prob)
    B.nmd_set_emitter(engine.ctx, 62, LINES, YIELDS, BETA)
    engine.run(62, 10 ** 7, 9001)
    gr, _, gs = engine.organs(62)
    led = engine.ledger(62)
    assert abs(_balance(led)) < 1e-9
    ph = oracle_phantom(orc, prob)
    tal, _ = orc.run(ph, 4 * 10 ** 6, 9002, emitter=(LINES, YIELDS, BETA))
    orr, os_ = orc.organ_mean_sigma(tal, prob.total_activity_bq)
    m = (gr > 0) & (orr > 0)
    z = (gr[m] - orr[m]) / np.sqrt((gr[m] * gs[m]) ** 2 + (orr[m] * os_[m]) ** 2)
    print("emitter organ z:", np.round(z, 2))
    assert m.sum() >= 10 and np.all(np.abs(z) <= 3.0)


def test_emitter_switch_and_validation(engine):
    prob = P.patient_phantom(shape=(50, 40, 40), voxel_mm=(12.0, 12.0, 18.0), seed=45)
    engine.set_problem(62, prob)
    for bad in (([1.2], [0.1], 0.1), ([0.1], [0.7, 0.5][:1] + [0.0], 0.1),
                ([0.1, 0.2], [0.6, 0.5], 0.1), ([0.1], [0.1], -0.1)):
        with pytest.raises((B.NmdError, ValueError)):
            B.nmd_set_emitter(engine.ctx, 62, *bad)
    iev = [75.0] * len(prob.materials)
    # lines above 511 keV and Compton electron transport exclude each other
    B.nmd_set_emitter(engine.ctx, 62, *EMITTERS["i131"])
    with pytest.raises(B.NmdError, match="NMD_E_UNSUPPORTED"):
        B.nmd_set_electrons(engine.ctx, 62, 0.2, iev)
    B.nmd_set_emitter(engine.ctx, 62)
    B.nmd_set_electrons(engine.ctx, 62, 0.2, iev)
    with pytest.raises(B.NmdError, match="NMD_E_UNSUPPORTED"):
        B.nmd_set_emitter(engine.ctx, 62, *EMITTERS["i131"])
    B.nmd_set_electrons(engine.ctx, 62, 0.0, None)
    B.nmd_set_emitter(engine.ctx, 62, LINES, YIELDS, BETA)
    with pytest.raises(B.NmdError, match="NMD_E_STATE"):
        B.nmd_set_positron(engine.ctx, 62, True, 0.5, iev)
    engine.run(62, 100_000, 3)
    led = engine.ledger(62)
    assert led["dep_beta"] == pytest.approx(100_000 * BETA, rel=1e-6)
    B.nmd_set_emitter(engine.ctx, 62)  # back to the photon pair
    assert engine.stats(62)["histories"] == 0
    engine.run(62, 100_000, 3)
    led = engine.ledger(62)
    assert led["dep_beta"] == 0.0
    assert led["emitted"] == pytest.approx(100_000 * 2 * 0.511, rel=1e-6)


def test_wide_and_pair_grid_phantoms_in_one_launch():
    """A 177Lu phantom (the pair's grid) and a 131I phantom (the wide grid)
    in one batched launch: each wave takes its phantom's grid, so each
    phantom gets exactly what its own launch gives."""
    def small(seed):
        return P.patient_phantom(shape=(50, 40, 40), voxel_mm=(12.0, 12.0, 18.0), seed=seed)

    def snap(eng, pid):
        s, s2, n = eng.tallies(pid)
        st = eng.stats(pid)
        for k in ("claims", "max_merged"):  # schedule-dependent
            st.pop(k)
        return s.cpu().numpy(), s2.cpu().numpy(), n, st, eng.ledger(pid)

    a, b = small(51), small(52)
    n, seed = 300_000, 93
    sep, bat = B.Engine(0), B.Engine(0)
    try:
        for e in (sep, bat):
            e.set_problem(1, a)
            e.set_problem(2, b)
            B.nmd_set_emitter(e.ctx, 1, *EMITTERS["lu177"])
            B.nmd_set_emitter(e.ctx, 2, *EMITTERS["i131"])
        sep.run(1, n, seed)
        sep.run(2, n, seed)
        B.nmd_run_histories(bat.ctx, -1, n, seed, None)
        for pid in (1, 2):
            x, y = snap(sep, pid), snap(bat, pid)
            assert x[2] == y[2] and x[3] == y[3]
            assert np.allclose(x[0], y[0], rtol=1e-12, atol=0)
            assert np.allclose(x[1], y[1], rtol=1e-12, atol=0)
            assert abs(_balance(y[4])) < 1e-9
    finally:
        sep.close()
        bat.close()
