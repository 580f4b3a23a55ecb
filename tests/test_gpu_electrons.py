"""Compton electrons above the cutoff on the device (Section 2.1 follows
electrons down to 200 keV): the electron walk of the transport kernel
against the oracle's electron option (oracle/nmd_oracle.c, pinned to ICRU
Report 37 in tests/test_oracle_electron.py), history by history on the same
random streams, and statistically against exact traversal."""
import numpy as np
import pytest

from conftest import ledger_balance, oracle_phantom
from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu
CUT = 0.2


def _iev(prob):
    return [P.MEAN_EXCITATION_EV[next(k for k in P.MATERIALS
                                      if tuple(P.MATERIALS[k][:2]) == tuple(m))]
            for m in prob.materials]


def _replay(engine, orc, pid, prob, n, seed, pencil=None):
    engine.set_problem(pid, prob)
    B.nmd_set_electrons(engine.ctx, pid, CUT, _iev(prob))
    t = engine.torch
    rec = t.zeros(n * 10, dtype=t.float64, device=engine.device)
    kw = {} if pencil is None else dict(source_kind=1, pencil_origin_cm=pencil[0],
                                        pencil_dir=pencil[1])
    engine.run(pid, n, seed, history_records=rec, **kw)
    g = rec.cpu().numpy().reshape(n, 10)
    tal, o = orc.run(oracle_phantom(orc, prob), n, seed, tracking=orc.TRACK_WOODCOCK, pid=pid,
                     history_records=True, electron_cutoff_mev=CUT,
                     mean_excitation_ev=_iev(prob), pencil=pencil)
    return g, o, tal


@pytest.mark.parametrize("name", ["slab", "patient"])
def test_electron_walk_replays_history_by_history(engine, orc, name):
    """Same draws, same photon events; the electrons leave the same energy in
    the same voxels (to the FP32 range tables and positions)."""
    if name == "slab":  # point source of pairs: the decay draws replay too
        prob, n, pencil = P.slab_phantom(n=64, voxel_mm=6.0), 30_000, None
    else:
        # the alias table and the oracle's CDF inversion map a word to
        # different voxels, so a spread-out activity map does not replay:
        # a pencil beam through the torso of a 4 mm patient instead
        prob, n = P.patient_phantom(shape=(240, 128, 128), voxel_mm=(4.0, 4.0, 4.0), seed=7), 20_000
        h = prob.voxel_cm
        pencil = ((0.0, 64.5 * h[1], 110.5 * h[2]), (1.0, 0.0, 0.0))
    g, o, tal = _replay(engine, orc, 40, prob, n, 19, pencil)
    same = np.all(g[:, [2, 3, 4, 5, 8]] == o[:, [2, 3, 4, 5, 8]], axis=1)
    assert same.mean() >= 0.995
    e_ok = np.abs(g[:, 0] - o[:, 0]) <= 1e-5 + 1e-5 * np.abs(o[:, 0])
    x_ok = np.abs(g[:, 1] - o[:, 1]) <= 1e-5 + 1e-5 * np.abs(o[:, 1])
    assert (same & e_ok & x_ok).mean() >= 0.995
    v_ok = (g[same, 7] == o[same, 7]) & (g[same, 6] == o[same, 6])
    assert v_ok.mean() >= 0.99, v_ok.mean()
    led = engine.ledger(40)
    assert abs(ledger_balance(led)) < 1e-9 and abs(ledger_balance(tal.ledger)) < 1e-9
    # the electrons do walk: histories deposit in more voxels than their
    # photon events alone
    ev = g[:, 2] + g[:, 3]
    assert (g[:, 7] > ev).sum() > 0.01 * n


def test_electrons_statistical_parity_on_the_patient(engine, orc):
    """Full-size patient with electrons against the exact-traversal oracle
    with electrons (independent streams): every organ within three combined
    sigma; the energy the walk moves changes small organs by percent."""
    prob = P.patient_phantom()
    engine.set_problem(41, prob)
    B.nmd_set_electrons(engine.ctx, 41, CUT, _iev(prob))
    engine.run(41, 10 ** 7, 7001)
    gr, _, gs = engine.organs(41)
    led = engine.ledger(41)
    assert abs(ledger_balance(led)) < 1e-9
    ph = oracle_phantom(orc, prob)
    tal, _ = orc.run(ph, 4 * 10 ** 6, 7002, electron_cutoff_mev=CUT,
                     mean_excitation_ev=_iev(prob))
    orr, os_ = orc.organ_mean_sigma(tal, prob.total_activity_bq)
    m = (gr > 0) & (orr > 0)
    z = (gr[m] - orr[m]) / np.sqrt((gr[m] * gs[m]) ** 2 + (orr[m] * os_[m]) ** 2)
    print("electrons organ z:", np.round(z, 2))
    assert m.sum() >= 20 and np.all(np.abs(z) <= 3.0)


def test_electron_model_switches_and_validation(engine):
    prob = P.slab_phantom(n=32, voxel_mm=8.0)
    iev = _iev(prob)
    engine.set_problem(42, prob)
    engine.run(42, 100_000, 3)
    s0, q0, _ = engine.tallies(42)
    B.nmd_set_electrons(engine.ctx, 42, CUT, iev)   # resets the tallies
    assert engine.stats(42)["histories"] == 0
    engine.run(42, 100_000, 3)
    s1, _, _ = engine.tallies(42)
    assert not np.array_equal(s0.cpu().numpy(), s1.cpu().numpy())
    # the total stays (few electrons leave this grid); the map spreads
    assert s1.sum().item() == pytest.approx(s0.sum().item(), rel=2e-3)
    B.nmd_set_electrons(engine.ctx, 42, 0.0)       # off again: the plain kernel
    engine.run(42, 100_000, 3)
    s2, q2, _ = engine.tallies(42)
    assert np.allclose(s2.cpu().numpy(), s0.cpu().numpy(), rtol=1e-12, atol=0)
    assert np.allclose(q2.cpu().numpy(), q0.cpu().numpy(), rtol=1e-12, atol=0)

    def status(*a):
        with pytest.raises(B.NmdError) as ei:
            B.nmd_set_electrons(engine.ctx, *a)
        return ei.value.status

    assert status(42, 0.5, iev) == -1          # above the largest Compton electron
    assert status(42, CUT, None) == -1
    assert status(42, CUT, [0.5] + iev[1:]) == -1
    assert status(64, CUT, iev) == -3          # no such phantom
