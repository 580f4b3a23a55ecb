"""Region tracking (nmd_set_tracking, NMD_TRACK_REGIONS): Woodcock steps
against the phantom's majorant inside the bounding box of its dense voxels
and a smaller one in the air around it.  The device replays the oracle's
region mode draw for draw; the doses agree in distribution with the
exact-traversal oracle; phantoms without an outer region draw exactly as
under global tracking, also inside a region-tracking launch; and the mode
cuts null collisions."""
import numpy as np
import pytest

from conftest import ledger_balance, oracle_phantom
from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu
INT_COLS = [2, 3, 4, 5, 8]  # n_compton, n_pe, n_rayleigh, n_steps, n_uniforms


def _replay(engine, orc, pid, prob, n, seed, pencil=None, **okw):
    engine.set_problem(pid, prob)
    B.nmd_set_tracking(engine.ctx, pid, "regions")
    t = engine.torch
    rec = t.zeros(n * 10, dtype=t.float64, device=engine.device)
    gkw = {}
    if pencil is not None:
        gkw.update(source_kind=1, pencil_origin_cm=pencil[0], pencil_dir=pencil[1])
        okw["pencil"] = pencil
    if "photons_per_decay" in okw:
        gkw["photons_per_decay"] = okw["photons_per_decay"]
    engine.run(pid, n, seed, history_records=rec, **gkw)
    g = rec.cpu().numpy().reshape(n, 10)
    ph = oracle_phantom(orc, prob)
    tal, o = orc.run(ph, n, seed, tracking=orc.TRACK_REGIONS, pid=pid, history_records=True,
                     **okw)
    return g, o, tal


def _check(g, o, frac=0.995):
    same = np.all(g[:, INT_COLS] == o[:, INT_COLS], axis=1)
    assert same.mean() >= frac, "identical event counts: %.5f" % same.mean()
    e_ok = np.abs(g[:, 0] - o[:, 0]) <= 1e-5 + 1e-5 * np.abs(o[:, 0])
    x_ok = np.abs(g[:, 1] - o[:, 1]) <= 1e-5 + 1e-5 * np.abs(o[:, 1])
    assert (same & e_ok & x_ok).mean() >= frac
    v_ok = (g[same, 7] == o[same, 7]) & (g[same, 6] == o[same, 6])
    assert v_ok.mean() >= frac


def test_regions_replay_slab(engine, orc):
    """Photon pairs in the slab's tissue block, which sits in air: photons
    leave the box, scatter in the air and come back."""
    prob = P.slab_phantom(n=64, voxel_mm=6.0)
    g, o, tal = _replay(engine, orc, 43, prob, 30_000, 31)
    _check(g, o)
    led = engine.ledger(43)
    assert abs(ledger_balance(led)) < 1e-9 and abs(ledger_balance(tal.ledger)) < 1e-9
    st = engine.stats(43)
    assert st["steps"] == tal.stats["steps"] or \
        abs(st["steps"] - tal.stats["steps"]) < 1e-3 * tal.stats["steps"]


def test_regions_replay_pencil_from_air(engine, orc):
    """A pencil beam that starts in the air beside the full-size patient,
    enters the box, crosses the body and leaves it."""
    prob = P.patient_phantom()
    h = prob.voxel_cm
    origin = (0.0, 128.5 * h[1], 250.5 * h[2])
    assert prob.density[250, 128, 0] < 0.01  # the beam starts in air
    g, o, _ = _replay(engine, orc, 44, prob, 20_000, 33, pencil=(origin, (1.0, 0.0, 0.0)))
    _check(g, o)
    assert (g[:, 2] > 0).mean() > 0.5


def test_regions_statistical_parity_patient(engine, orc):
    """Organ doses of the patient under region tracking against the
    exact-traversal oracle (independent tracking, sampler and streams):
    every organ within three combined standard errors; fewer null
    collisions than global tracking of the same decays."""
    prob = P.patient_phantom()
    n = 10 ** 7
    engine.set_problem(46, prob)
    B.nmd_set_tracking(engine.ctx, 46, "regions")
    engine.run(46, n, 1001, photons_per_decay=2)
    gr, _, gs = engine.organs(46)
    st_r = engine.stats(46)
    assert abs(ledger_balance(engine.ledger(46))) < 1e-9
    ph = oracle_phantom(orc, prob)
    tal, _ = orc.run(ph, 4 * 10 ** 6, 2002, photons_per_decay=2)
    orr, os_ = orc.organ_mean_sigma(tal, prob.total_activity_bq)
    m = (gr > 0) & (orr > 0)
    z = (gr[m] - orr[m]) / np.sqrt((gr[m] * gs[m]) ** 2 + (orr[m] * os_[m]) ** 2)
    print("regions organ z:", np.round(z, 2))
    assert m.sum() >= 10 and np.all(np.abs(z) <= 3.0)
    B.nmd_set_tracking(engine.ctx, 46, "global")
    B.nmd_reset_tallies(engine.ctx, 46)
    engine.run(46, n, 1001, photons_per_decay=2)
    st_g = engine.stats(46)
    print("nulls per decay: global %.3f, regions %.3f" % (st_g["nulls"] / n, st_r["nulls"] / n))
    assert st_r["nulls"] < 0.6 * st_g["nulls"]
    assert st_r["histories"] == st_g["histories"] == n


def _small(seed):
    return P.patient_phantom(shape=(50, 40, 40), voxel_mm=(12.0, 12.0, 18.0), seed=seed)


def _snap(eng, pid):
    s, s2, n = eng.tallies(pid)
    st = eng.stats(pid)
    # schedule-dependent counters; and the global kernel gathers a record
    # ahead that the region kernel reads only when its step comes
    for k in ("claims", "max_merged", "gathers"):
        st.pop(k)
    return s.cpu().numpy(), s2.cpu().numpy(), n, st


def test_regions_batched_with_global_phantom():
    """A batched launch that holds a region-tracking phantom runs the
    region kernel for every phantom: a phantom in global mode there draws
    exactly as in its own global launch, and the region phantom as in its
    own region launch."""
    a, b = _small(41), _small(42)
    n, seed = 300_000, 91
    sep = B.Engine(0)
    bat = B.Engine(0)
    try:
        for e in (sep, bat):
            e.set_problem(1, a)
            e.set_problem(2, b)
            B.nmd_set_tracking(e.ctx, 2, "regions")
        sep.run(1, n, seed)
        sep.run(2, n, seed)
        B.nmd_run_histories(bat.ctx, -1, n, seed, None)
        for pid in (1, 2):
            x, y = _snap(sep, pid), _snap(bat, pid)
            assert x[2] == y[2] and x[3] == y[3]
            assert np.allclose(x[0], y[0], rtol=1e-12, atol=0)
            assert np.allclose(x[1], y[1], rtol=1e-12, atol=0)
        # the region phantom really took fewer steps than it would globally
        glob = B.Engine(0)
        try:
            glob.set_problem(2, b)
            glob.run(2, n, seed)
            assert sep.stats(2)["nulls"] < glob.stats(2)["nulls"]
        finally:
            glob.close()
    finally:
        sep.close()
        bat.close()


def test_regions_one_region_phantom_draws_as_global(engine):
    """A water cube has no outer region (its box is the whole grid): region
    tracking leaves every draw as under global tracking."""
    prob = P.water_point_source(n=32, voxel_mm=2.0)
    engine.set_problem(47, prob)
    engine.run(47, 200_000, 5, photons_per_decay=1)
    g = _snap(engine, 47)
    B.nmd_set_tracking(engine.ctx, 47, "regions")
    B.nmd_reset_tallies(engine.ctx, 47)
    engine.run(47, 200_000, 5, photons_per_decay=1)
    r = _snap(engine, 47)
    assert g[2] == r[2] and g[3] == r[3]
    assert np.allclose(g[0], r[0], rtol=1e-12, atol=0)


def test_regions_switch_validation_and_graphs(engine):
    """Errors, and graphs captured before a switch refuse to launch."""
    prob = _small(43)
    engine.set_problem(48, prob)
    with pytest.raises(B.NmdError, match="NMD_E_INVALID"):
        B.nmd_set_tracking(engine.ctx, 48, 2)
    with pytest.raises(B.NmdError, match="NMD_E_STATE"):
        B.nmd_set_tracking(engine.ctx, 49, "regions")
    g = B.nmd_graph_create(engine.ctx, 48, 10_000, 3, None, None, None)
    try:
        B.nmd_graph_launch(engine.ctx, g)
        B.nmd_set_tracking(engine.ctx, 48, "regions")
        with pytest.raises(B.NmdError, match="NMD_E_STATE"):
            B.nmd_graph_launch(engine.ctx, g)
    finally:
        B.nmd_graph_destroy(g)
    # re-registering returns the phantom to global tracking
    engine.set_problem(48, prob)
    engine.run(48, 100_000, 4)
    a = _snap(engine, 48)
    engine.set_problem(48, prob)
    B.nmd_set_tracking(engine.ctx, 48, "global")
    engine.run(48, 100_000, 4)
    b = _snap(engine, 48)
    assert a[3] == b[3]
