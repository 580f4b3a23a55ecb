"""The seeded input generators: determinism, structure and normalisation."""
import numpy as np
import pytest

from paper_2111_11687_amd import phantoms as P


def test_water_point_source():
    p = P.water_point_source(n=64)
    assert p.shape == (64, 64, 64) and p.voxel_mm == (2.0, 2.0, 2.0)
    assert p.activity.sum() == 1.0 and p.activity[32, 32, 32] == 1.0
    assert p.photons_per_decay == 1 and p.n_organs == 32
    assert set(np.unique(p.material)) == {0}
    assert p.label[32, 32, 32] == 1 and p.label[32, 32, 63] == 32


def test_slab_phantom_structure_and_determinism():
    a, b = P.slab_phantom(), P.slab_phantom()
    for f in ("density", "material", "label", "activity"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert a.shape == (128, 128, 128) and a.voxel_mm == (3.0, 3.0, 3.0)
    counts = np.bincount(a.material.ravel(), minlength=4)
    assert np.all(counts > 0)
    assert np.allclose(np.unique(a.density), [0.0012, 0.26, 1.0, 1.85], rtol=1e-6)
    z0, z1 = a.extra["slab_z"]
    assert 64 + 6 <= z0 and z1 - z0 >= 15
    assert a.activity[64, 64, 64] == 1.0 and a.activity.sum() == 1.0
    assert a.material[64, 64, 64] == 2  # source in soft tissue


def test_patient_phantom_organs_and_activity():
    p = P.patient_phantom(shape=(160, 128, 128), voxel_mm=(4.0, 4.0, 6.0), seed=3)
    assert p.n_organs == 28 and len(p.organ_names) == 28
    cnt = np.bincount(p.label.ravel(), minlength=29)
    assert np.all(cnt[1:] > 0), "every organ present"
    assert set(np.unique(p.material)) == {0, 1, 2, 3}
    assert np.all(p.activity[p.label == 0] == 0)
    assert np.all(p.activity[p.label > 0] >= 0)
    vol = np.prod(p.voxel_cm)
    assert p.activity.astype(np.float64).sum() * vol == pytest.approx(p.total_activity_bq,
                                                                        rel=1e-5, abs=0)
    assert p.total_activity_bq == pytest.approx(8.0 * 3.7e7 * 0.5 ** (60 / 109.77))
    lungs = (p.label == P.ORGANS.index("Lung_Left") + 1)
    assert np.all(p.density[lungs] == np.float32(0.26))
    q = P.patient_phantom(shape=(160, 128, 128), voxel_mm=(4.0, 4.0, 6.0), seed=3)
    assert np.array_equal(p.activity, q.activity) and np.array_equal(p.label, q.label)


def test_batch_sizes():
    ps = P.batch_phantoms(n=3)
    for p in ps:
        nz, ny, nx = p.shape
        assert 64 <= nx <= 192 and 64 <= ny <= 192 and 64 <= nz <= 256
        assert p.voxel_mm[0] in (2.0, 3.0, 4.0)
