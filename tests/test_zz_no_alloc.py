"""nmd_organ_mean_map_noalloc (for callers that cannot allocate) against
nmd_organ_mean_map on the same maps, through the C ABI: two calls in a row,
the second on a smaller phantom with fewer labels, so that the first call's
sums left in the shared device scratch must not reach the second's result."""
import numpy as np
import pytest

from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu


def _map(engine, prob, seed):
    rng = np.random.default_rng(seed)
    m = rng.gamma(2.0, 1e-7, size=prob.shape)
    return engine.torch.from_numpy(m).to(engine.device), m


def _numpy_means(prob, m):
    lab = prob.label.ravel()
    s = np.bincount(lab, weights=m.ravel(), minlength=prob.n_organs + 1)
    c = np.bincount(lab, minlength=prob.n_organs + 1)
    return np.where(c[1:] > 0, s[1:] / np.maximum(c[1:], 1), 0.0)


def test_noalloc_organ_means_equal_the_allocating_call():
    eng = B.Engine(0)
    try:
        big = P.patient_phantom(shape=(80, 64, 64), voxel_mm=(8.0, 8.0, 12.0), seed=9)
        small = P.slab_phantom(n=24, voxel_mm=12.0)
        assert small.n_organs < big.n_organs and small.nvox < big.nvox
        eng.set_problem(1, big, with_activity=False)
        eng.set_problem(2, small, with_activity=False)
        for pid, prob, seed in ((1, big, 11), (2, small, 12)):
            dmap, hmap = _map(eng, prob, seed)
            na = B.nmd_organ_mean_map_noalloc(eng.ctx, pid, dmap, prob.n_organs)
            ref = B.nmd_organ_mean_map(eng.ctx, pid, dmap, prob.n_organs)
            assert np.allclose(na, ref, rtol=1e-12, atol=0)
            assert np.allclose(na, _numpy_means(prob, hmap), rtol=1e-12, atol=0)
            assert (na > 0).sum() >= min(prob.n_organs, 10)
        # a phantom without labels is refused, as by the allocating call
        eng.set_problem(3, small, with_activity=False)
        B.nmd_set_phantom(eng.ctx, 3, eng.inputs[3]["density"], eng.inputs[3]["material"],
                          None, 0, small.materials, small.voxel_mm)
        with pytest.raises(B.NmdError) as ei:
            B.nmd_organ_mean_map_noalloc(eng.ctx, 3, dmap, 0)
        assert ei.value.status == -3
    finally:
        eng.close()
