"""Device samplers against the oracle through the C ABI: Philox words and
uniforms bit for bit, the Marsaglia, Klein-Nishina and Thomson samplers draw
for draw (FP32 against FP64), the alias-table decay sampler against the
activity distribution, and the FP32 majorant against every attenuation
coefficient it must bound."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2111_11687_amd import binding as B
from paper_2111_11687_amd import phantoms as P

pytestmark = pytest.mark.gpu
MEC2 = 0.51099895


def _dev(engine, n, dtype=None):
    t = engine.torch
    return t.zeros(n, dtype=dtype or t.float64, device=engine.device)


@pytest.mark.parametrize("seed", [0, 12345, 2 ** 40 + 17, 2 ** 64 - 1])
def test_philox_words_bit_exact(engine, orc, seed):
    n = 4099  # several blocks of 256 plus a ragged tail
    out = _dev(engine, 4 * n)
    B.nmd_debug_sample(engine.ctx, 0, 0.511, n, seed, out)
    g = out.cpu().numpy().reshape(n, 4)
    assert np.array_equal(g, orc.sample("raw", n, seed=seed))


def test_uniforms_bit_exact(engine, orc):
    n = 100_003
    out = _dev(engine, n)
    B.nmd_debug_sample(engine.ctx, 1, 0.511, n, 99, out)
    assert np.array_equal(out.cpu().numpy(), orc.sample("uniform", n, seed=99))


def test_marsaglia_replay(engine, orc):
    n = 200_000
    out = _dev(engine, 3 * n)
    B.nmd_debug_sample(engine.ctx, 2, 0.511, n, 5, out)
    g = out.cpu().numpy().reshape(n, 3)
    o = orc.sample("marsaglia", n, seed=5)
    # FP32 rounding of 1 - s is amplified by sqrt(1 - s) near the pole
    # (1 - s = (1 + d_z) / 2): allow the derived bound there
    tol = 3e-6 + 1.2e-7 / np.sqrt(np.maximum((1.0 + o[:, 2]) / 2.0, 1e-14))
    close = np.all(np.abs(g - o) <= tol[:, None], axis=1)
    assert close.mean() > 0.99999  # a draw on the s = 1 edge may flip in FP32
    assert np.allclose(np.linalg.norm(g, axis=1), 1.0, atol=3e-6)


@pytest.mark.parametrize("e", [0.511, 0.2, 0.05, 0.012])
def test_klein_nishina_replay_and_chi2(engine, orc, e):
    n = 1_000_000
    out = _dev(engine, 2 * n)
    B.nmd_debug_sample(engine.ctx, 3, e, n, 17, out)
    g = out.cpu().numpy().reshape(n, 2)
    o = orc.sample("butcher", n, seed=17, e_mev=e)
    d = np.abs(g - o).max(axis=1)
    assert (d < 5e-5).mean() > 0.999
    # the device distribution itself against the integrated KN cross section
    k = e / MEC2

    def dsig(c):
        p = 1.0 / (1.0 + k * (1.0 - c))
        return p * p * (p + 1.0 / p - (1.0 - c * c))

    edges = np.linspace(-1, 1, 51)
    tot = integrate.quad(dsig, -1, 1, epsrel=1e-12)[0]
    mass = np.array([integrate.quad(dsig, a, b, epsrel=1e-12)[0]
                     for a, b in zip(edges[:-1], edges[1:])]) / tot
    obs = np.histogram(np.clip(g[:, 1], -1, 1), bins=edges)[0]
    exp = mass * n
    assert stats.chi2.sf(((obs - exp) ** 2 / exp).sum(), 49) > 1e-3


def test_thomson_replay(engine, orc):
    n = 300_000
    out = _dev(engine, n)
    B.nmd_debug_sample(engine.ctx, 5, 0.511, n, 23, out)
    g = out.cpu().numpy()
    o = orc.sample("thomson", n, seed=23)
    assert np.abs(g - o).max() < 2e-6


def test_alias_sampler_matches_activity(engine):
    prob = P.patient_phantom(shape=(40, 32, 32), voxel_mm=(16.0, 16.0, 24.0), seed=7)
    engine.set_problem(5, prob)
    n = 4_000_000
    out = engine.torch.zeros(n, dtype=engine.torch.int32, device=engine.device)
    B.nmd_debug_sample_source(engine.ctx, 5, n, 31, out)
    v = out.cpu().numpy().astype(np.int64)
    a = prob.activity.ravel().astype(np.float64)
    assert v.min() >= 0 and v.max() < a.size
    assert np.all(a[v] > 0)  # never a voxel without activity
    p = a / a.sum()
    obs = np.bincount(v, minlength=a.size)
    nz = p > 0
    exp = p[nz] * n
    # pool voxels with small expectations to keep the chi-square valid
    order = np.argsort(exp)
    e_s, o_s = exp[order], obs[nz][order]
    cuts = np.searchsorted(np.cumsum(e_s), np.arange(20.0, e_s.sum(), 20.0))
    eb = np.add.reduceat(e_s, np.unique(np.r_[0, cuts[cuts < len(e_s)]]))
    ob = np.add.reduceat(o_s, np.unique(np.r_[0, cuts[cuts < len(e_s)]]))
    chi2 = ((ob - eb) ** 2 / eb).sum()
    assert stats.chi2.sf(chi2, len(eb) - 1) > 1e-3


def test_majorant_bounds_every_material(engine, orc):
    prob = P.patient_phantom(shape=(40, 32, 32), voxel_mm=(16.0, 16.0, 24.0), seed=7)
    engine.set_problem(6, prob)
    t = engine.torch
    e = np.exp(np.linspace(math.log(0.0101), math.log(0.511), 100_000)).astype(np.float32)
    et = t.from_numpy(e).to(engine.device)
    out = t.zeros(2 * len(e), dtype=t.float32, device=engine.device)
    B.nmd_debug_xs(engine.ctx, 6, et, out)
    r = out.cpu().numpy().reshape(-1, 2)
    maj, mu = r[:, 0].astype(np.float64), r[:, 1].astype(np.float64)
    assert np.all(maj >= mu)
    assert (maj / mu - 1).max() < 0.02  # a tight bound
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm)
    for x in e[::9973]:
        assert maj[np.searchsorted(e, x)] == pytest.approx(ph.majorant(float(x)), rel=2e-5)
