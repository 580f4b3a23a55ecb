"""Scoring kernels on seeded synthetic tallies (Eq. 1 per voxel, Eq. 2 and
Eq. 3 per organ) against the oracle's FP64 formulas; schedule invariance
(chunk size, grid size, batched against separate launches, resumed against
one long run) as a race detector; error paths of the C ABI."""
import numpy as np
import pytest

from conftest import oracle_phantom
from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu


def _small(seed=9):
    return P.patient_phantom(shape=(60, 48, 48), voxel_mm=(10.0, 10.0, 16.0), seed=seed)


def test_finalize_and_organ_reduce_on_synthetic_tallies(engine, orc):
    prob = _small()
    engine.set_problem(30, prob)
    t = engine.torch
    rng = np.random.default_rng(30)
    N = 123457
    S = rng.gamma(0.5, 3.0, size=prob.shape) * (rng.random(prob.shape) < 0.8)
    S2 = S * S / N * rng.uniform(1.0, 50.0, size=prob.shape)
    S2[rng.random(prob.shape) < 0.01] = 0.0  # negative variance estimates clamp to 0
    B.nmd_set_tallies(engine.ctx, 30, t.from_numpy(S).to(engine.device),
                      t.from_numpy(S2).to(engine.device), N)
    rate, rel = engine.dose(30)
    ph = oracle_phantom(orc, prob)
    tal = orc.Tally(ph)
    tal.S[...] = S
    tal.S2[...] = S2
    tal.n_decays = N
    od, oe = orc.finalize(ph, tal, prob.total_activity_bq)
    gd, ge = rate.cpu().numpy(), rel.cpu().numpy()
    assert np.allclose(gd, od, rtol=1e-13, atol=0)
    assert np.allclose(ge, oe, rtol=1e-12, atol=1e-300)
    assert np.array_equal(gd == 0, od == 0)
    r, e3, _ = engine.organs(30, sigma=False)
    orr, oe3 = orc.organ_stats(ph, od, oe)
    assert np.allclose(r, orr, rtol=1e-12, atol=0)
    assert np.allclose(e3, oe3, rtol=1e-12, atol=0)


def _state(engine, pid):
    s, s2, n = engine.tallies(pid)
    st = engine.stats(pid)
    st.pop("claims")
    st.pop("max_merged")
    return s.cpu().numpy(), s2.cpu().numpy(), n, st, engine.ledger(pid)


def _same(a, b):
    assert a[2] == b[2]
    assert a[3] == b[3]  # integer counters exactly
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=0)
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=0)
    for k in a[4]:
        assert a[4][k] == pytest.approx(b[4][k], rel=1e-12)


def test_schedule_invariance_chunk_and_grid(engine):
    prob = _small()
    engine.set_problem(31, prob)
    n = 300_001
    engine.run(31, n, 77)
    ref = _state(engine, 31)
    for kw in (dict(chunk=64), dict(chunk=4096, grid_blocks=37), dict(chunk=1, grid_blocks=4)):
        B.nmd_reset_tallies(engine.ctx, 31)
        engine.run(31, n, 77, **kw)
        _same(_state(engine, 31), ref)


def test_resume_equals_one_long_run(engine):
    prob = _small()
    engine.set_problem(32, prob)
    engine.run(32, 500_000, 5)
    ref = _state(engine, 32)
    B.nmd_reset_tallies(engine.ctx, 32)
    engine.run(32, 123_456, 5)
    engine.run(32, 500_000 - 123_456, 5, chunk=100)
    _same(_state(engine, 32), ref)


def test_batched_launch_equals_separate_launches():
    """One persistent launch over several phantoms of uneven size gives each
    phantom exactly what its own launch gives (random streams depend only on
    seed, phantom and history)."""
    probs = [_small(9), P.water_point_source(n=40, voxel_mm=3.0), P.slab_phantom(n=48)]
    ids = [3, 17, 40]
    n = 200_000
    eng = B.Engine(0)
    try:
        refs = []
        for i, p in zip(ids, probs):
            eng.set_problem(i, p)
            eng.run(i, n, 8)
            refs.append(_state(eng, i))
        B.nmd_reset_tallies(eng.ctx, -1)
        eng.run(-1, n, 8, chunk=512)
        for i, r in zip(ids, refs):
            _same(_state(eng, i), r)
    finally:
        eng.close()


def _full(engine, pid, n_organs):
    """Everything a run changes: tallies, counters, ledger, organ sums."""
    s = _state(engine, pid)
    r, e3, sig = engine.organs(pid)
    return s + (r, e3, sig, B.nmd_get_organ_score(engine.ctx, pid, n_organs))


def _same_full(a, b, exact=False):
    if exact:
        # the sums themselves bit for bit; the organ reduction of Eq. 2 and
        # Eq. 3 runs again, with its FP64 atomics in another order
        assert a[2] == b[2] and a[3] == b[3] and a[4] == b[4]
        for i in (0, 1, 7, 8):
            assert np.array_equal(a[i], b[i])
        for i in (5, 6):
            assert np.allclose(a[i], b[i], rtol=1e-13, atol=0)
        return
    _same(a[:5], b[:5])
    for x, y in zip(a[5:], b[5:]):
        assert np.allclose(x, y, rtol=1e-10, atol=0)


def test_abort_hook_leaves_the_phantom_unchanged(engine):
    """A run stopped by the abort hook returns NMD_E_ABORTED and leaves the
    tallies, organ sums, ledger, counters and history count exactly as they
    were; the next run then continues the streams as if it never happened."""
    prob = _small()
    engine.set_problem(33, prob)
    engine.run(33, 200_000, 3)
    before = _full(engine, 33, prob.n_organs)
    with pytest.raises(B.NmdError) as ei:
        engine.run(33, 10 ** 6, 3, chunk=1000, abort_after_chunks=5)
    assert ei.value.status == -6
    _same_full(_full(engine, 33, prob.n_organs), before, exact=True)
    # an armed hook that does not fire commits the run like a plain one
    engine.run(33, 100_000, 3, chunk=1000, abort_after_chunks=10 ** 6)
    engine.run(33, 100_000, 3)
    got = _full(engine, 33, prob.n_organs)
    engine.set_problem(33, prob)  # the phantom id is part of the streams
    engine.run(33, 400_000, 3)
    _same_full(got, _full(engine, 33, prob.n_organs))


def test_set_tallies_voids_the_organ_sigma(engine):
    """Voxel sums restored by nmd_set_tallies keep Eq. 1-3 available, but the
    per-history organ sums no longer cover the N histories: the organ-mean
    sigma and the organ score are refused rather than divided by the wrong N."""
    prob = _small()
    engine.set_problem(35, prob)
    engine.run(35, 100_000, 4)
    r0, e0, _ = engine.organs(35)
    s, s2, n = engine.tallies(35)
    B.nmd_set_tallies(engine.ctx, 35, s, s2, n)
    r1, e1, _ = engine.organs(35, sigma=False)
    assert np.allclose(r1, r0, rtol=1e-13, atol=0) and np.allclose(e1, e0, rtol=1e-12, atol=0)
    for fn in (lambda: engine.organs(35),
               lambda: B.nmd_get_organ_score(engine.ctx, 35, prob.n_organs)):
        with pytest.raises(B.NmdError) as ei:
            fn()
        assert ei.value.status == -3
    B.nmd_reset_tallies(engine.ctx, 35)
    engine.run(35, 1000, 4)
    engine.organs(35)  # covered again after a reset


def test_save_load_equals_one_long_run(engine, tmp_path):
    """Save after N1 histories, load into the phantom registered afresh, run N2
    more with the same seed: tallies, organ rates, organ sigma, ledger and
    counters equal one run of N1 + N2 (up to the order of FP64 atomics)."""
    prob = _small()
    path = str(tmp_path / "ckpt.nmd")
    engine.set_problem(36, prob)
    engine.run(36, 150_000, 6)
    B.nmd_save(engine.ctx, 36, path)
    # a fresh registration of the same id (its random streams are keyed by
    # the id), restored from the file
    engine.set_problem(36, prob)
    B.nmd_load(engine.ctx, 36, path)
    engine.run(36, 250_000, 6)
    got = _full(engine, 36, prob.n_organs)
    engine.set_problem(36, prob)
    engine.run(36, 400_000, 6)
    ref = _full(engine, 36, prob.n_organs)
    _same_full(got, ref)
    assert got[2] == 400_000 and (got[7] > 0).sum() >= 20  # the organs this phantom holds


def test_load_rejects_other_phantoms_and_damaged_files(engine, tmp_path):
    prob = _small()
    path = str(tmp_path / "ckpt.nmd")
    engine.set_problem(38, prob)
    engine.run(38, 50_000, 7)
    B.nmd_save(engine.ctx, 38, path)
    before = _full(engine, 38, prob.n_organs)

    def status(*a):
        with pytest.raises(B.NmdError) as ei:
            B.nmd_load(engine.ctx, *a)
        return ei.value.status

    other = _small(seed=10)  # same shape, other organs and activity
    engine.set_problem(39, other)
    assert status(39, path) == -3
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0x40
    bad = str(tmp_path / "bad.nmd")
    open(bad, "wb").write(bytes(raw))
    assert status(38, bad) == -1
    open(bad, "wb").write(bytes(raw[:1000]))
    assert status(38, bad) == -1
    assert status(38, str(tmp_path / "missing.nmd")) == -1
    _same_full(_full(engine, 38, prob.n_organs), before, exact=True)


def test_error_paths(engine):
    t = engine.torch
    dev = engine.device
    ctx = engine.ctx
    rho = t.ones((4, 4, 4), dtype=t.float32, device=dev)
    mat = t.zeros((4, 4, 4), dtype=t.uint8, device=dev)
    lab = t.ones((4, 4, 4), dtype=t.uint8, device=dev)
    mats = [(7.4, 0.55)]

    def status(fn, *a):
        with pytest.raises(B.NmdError) as ei:
            fn(*a)
        return ei.value.status

    bad = rho.clone()
    bad[1, 2, 3] = -1.0
    assert status(B.nmd_set_phantom, ctx, 50, bad, mat, lab, 1, mats, (1, 1, 1)) == -1
    bad = rho.clone()
    bad[0, 0, 0] = float("nan")
    assert status(B.nmd_set_phantom, ctx, 50, bad, mat, lab, 1, mats, (1, 1, 1)) == -1
    assert status(B.nmd_set_phantom, ctx, 50, rho, mat + 1, lab, 1, mats, (1, 1, 1)) == -1
    assert status(B.nmd_set_phantom, ctx, 50, rho, mat, lab + 1, 1, mats, (1, 1, 1)) == -1
    assert status(B.nmd_set_phantom, ctx, 64, rho, mat, lab, 1, mats, (1, 1, 1)) == -1
    assert status(B.nmd_set_phantom, ctx, 50, rho, mat, lab, 1, mats, (0, 1, 1)) == -1
    B.nmd_set_phantom(ctx, 50, rho, mat, lab, 1, mats, (1, 1, 1))
    assert status(B.nmd_run_histories, ctx, 50, 10, 1, None) == -3  # no activity yet
    act = t.zeros((4, 4, 4), dtype=t.float32, device=dev)
    assert status(B.nmd_set_activity, ctx, 50, act, 0.0) == -1  # all zero
    act[2, 2, 2] = 1.0
    B.nmd_set_activity(ctx, 50, act, 0.0)
    o = B.nmd_run_opts_default()
    o.photon_cutoff_mev = 0.0
    assert status(B.nmd_run_histories, ctx, 50, 10, 1, o) == -1
    o = B.nmd_run_opts_default()
    o.source_kind = 1
    o.pencil_origin_cm[0] = 5.0  # outside the 0.4 cm grid
    assert status(B.nmd_run_histories, ctx, 50, 10, 1, o) == -1
    assert status(B.nmd_get_dose, ctx, 51, rho, None) == -3
    # more distinct (material, density) pairs than u8 records can index
    many = t.linspace(0.5, 2.0, 400, device=dev, dtype=t.float32).reshape(4, 10, 10)
    assert status(B.nmd_set_phantom, ctx, 52, many, t.zeros_like(many, dtype=t.uint8), None,
                  0, mats, (1, 1, 1)) == -7
    # the context is still usable after the errors
    B.nmd_run_histories(ctx, 50, 1000, 1, None)
    led = B.nmd_get_ledger(ctx, 50)
    assert led["emitted"] == pytest.approx(2 * 1000 * np.float32(0.511), rel=1e-12)
