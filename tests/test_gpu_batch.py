"""Batched runs: graph capture and replay, the online chunk autotuner, and a
persistent launch over several phantoms of uneven size.  Random streams
depend only on (seed, phantom, history), so a captured run replayed k times,
a tuned run and a batched run must reproduce the plain runs up to the order
of the FP64 atomic additions."""
import numpy as np
import pytest

from conftest import ledger_balance
from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu


def _small(seed):
    return P.patient_phantom(shape=(50, 40, 40), voxel_mm=(12.0, 12.0, 18.0), seed=seed)


def _snap(eng, pid):
    s, s2, n = eng.tallies(pid)
    st = eng.stats(pid)
    for k in ("claims", "max_merged"):
        st.pop(k)
    return s.cpu().numpy(), s2.cpu().numpy(), n, st


def _close(a, b):
    assert a[2] == b[2] and a[3] == b[3]
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=0)
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=0)


def test_graph_replays_equal_eager_runs():
    prob = _small(21)
    n, seed, reps = 300_000, 77, 3
    eager = B.Engine(0)
    graph_eng = B.Engine(0)
    try:
        eager.set_problem(1, prob)
        graph_eng.set_problem(1, prob)
        t = graph_eng.torch
        rate_g = t.empty(prob.shape, dtype=t.float64, device=graph_eng.device)
        rel_g = t.empty_like(rate_g)
        g = B.nmd_graph_create(graph_eng.ctx, 1, n, seed, None, rate_g, rel_g)
        try:
            for k in range(reps):
                eager.run(1, n, seed)
                rate_e, rel_e = eager.dose(1)
                org_e = eager.organs(1)
                B.nmd_graph_launch(graph_eng.ctx, g)
                # eager work of the program between replays
                _ = (t.ones(1000, device=graph_eng.device) * 2).sum().item()
                graph_eng.sync()
                _close(_snap(graph_eng, 1), _snap(eager, 1))
                assert np.allclose(rate_g.cpu().numpy(), rate_e.cpu().numpy(), rtol=1e-12, atol=0)
                assert np.allclose(rel_g.cpu().numpy(), rel_e.cpu().numpy(), rtol=1e-9, atol=0)
                org_g = B.nmd_read_organ_dose(graph_eng.ctx, 1, prob.n_organs)
                for x, y in zip(org_g, org_e):
                    assert np.allclose(x, y, rtol=1e-10, atol=0)
                assert B.nmd_get_run_stats(graph_eng.ctx, 1)["histories"] == (k + 1) * n
            # re-registering a phantom invalidates the graph
            graph_eng.set_problem(1, prob)
            with pytest.raises(B.NmdError) as ei:
                B.nmd_graph_launch(graph_eng.ctx, g)
            assert ei.value.status == -3
        finally:
            B.nmd_graph_destroy(g)
    finally:
        eager.close()
        graph_eng.close()


def test_autotuned_chunk_reproduces_fixed_chunk():
    prob = _small(22)
    n = (1 << 22) + 12345  # large enough to tune on, with a ragged tail
    eng = B.Engine(0)
    try:
        eng.set_problem(2, prob)
        eng.run(2, n, 5, chunk=512)
        ref = _snap(eng, 2)
        B.nmd_reset_tallies(eng.ctx, 2)
        eng.run(2, n, 5)  # chunk 0: tuned on this run
        chunk, grid = B.nmd_get_last_launch(eng.ctx)
        assert chunk in (128, 256, 512, 1024, 2048, 4096) and grid > 0
        _close(_snap(eng, 2), ref)
        # the tuned value is reused without tuning again
        B.nmd_reset_tallies(eng.ctx, 2)
        eng.run(2, n, 5)
        assert B.nmd_get_last_launch(eng.ctx)[0] == chunk
        _close(_snap(eng, 2), ref)
    finally:
        eng.close()


def test_batched_graph_over_uneven_phantoms():
    probs = P.batch_phantoms(n=6, first_seed=4000)
    n = 100_000
    ref_eng = B.Engine(0)
    eng = B.Engine(0)
    try:
        refs = {}
        for i, p in enumerate(probs):
            ref_eng.set_problem(i, p)
            ref_eng.run(i, 2 * n, 9)
            refs[i] = _snap(ref_eng, i)
            eng.set_problem(i, p)
        g = B.nmd_graph_create(eng.ctx, -1, n, 9)
        try:
            B.nmd_graph_launch(eng.ctx, g)
            eng.sync()
            B.nmd_graph_launch(eng.ctx, g)
            eng.sync()
        finally:
            B.nmd_graph_destroy(g)
        for i, p in enumerate(probs):
            _close(_snap(eng, i), refs[i])
            assert abs(ledger_balance(eng.ledger(i))) < 1e-9
            r, _, _ = B.nmd_read_organ_dose(eng.ctx, i, p.n_organs)
            r_eager, _, _ = eng.organs(i)
            assert np.allclose(r, r_eager, rtol=1e-12, atol=0)
    finally:
        ref_eng.close()
        eng.close()
