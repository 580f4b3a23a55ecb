"""Pins of the oracle's primitives against values fixed outside the oracle:
published generator outputs, numerical integration of the cross sections,
closed-form distributions and invariants."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats

RE = 2.8179403262e-13
MEC2 = 0.51099895
NA = 6.02214076e23


# ---------------------------------------------------------------- Philox
def test_philox_known_answers(orc):
    # Known-answer vectors published with the Random123 library (Salmon et
    # al., SC'11) for Philox4x32-10.
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert list(orc.philox(ctr, key)) == want


_RR_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char **argv) {
  unsigned long long seed = strtoull(argv[1], 0, 0), sub = strtoull(argv[2], 0, 0),
                     off = strtoull(argv[3], 0, 0);
  int n = atoi(argv[4]);
  rocrand_state_philox4x32_10 s;
  rocrand_init(seed, sub, off, &s);
  for (int i = 0; i < n; ++i) printf("%u\n", rocrand(&s));
}
"""


def _rocrand_words(tmp_path, seed, sub, off, n):
    exe = tmp_path / "rr"
    if not exe.exists():
        src = tmp_path / "rr.cpp"
        src.write_text(_RR_SRC)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__",
                               "-I/opt/rocm/include", str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe), str(seed), str(sub), str(off), str(n)])
    return [int(x) for x in out.split()]


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h")
                    or shutil.which("g++") is None, reason="rocRAND headers not installed")
def test_philox_matches_rocrand_host(orc, tmp_path):
    """The per-history stream (counter = (block, hid_lo, hid_hi, pid), key =
    seed) equals rocRAND's Philox4x32-10 started at subsequence (pid, hid_hi)
    and offset 4 * (hid_lo, block)."""
    for seed, hid, pid in [(12345, 0, 0), (2 ** 40 + 7, 123456789, 3), (1, 2 ** 33 + 5, 63)]:
        hid_lo, hid_hi = hid & 0xFFFFFFFF, hid >> 32
        sub = (pid << 32) | hid_hi
        off = 4 * (hid_lo << 32)
        want = _rocrand_words(tmp_path, seed, sub, off, 12)
        got = []
        for blk in range(3):
            got += list(orc.philox([blk, hid_lo, hid_hi, pid],
                                   [seed & 0xFFFFFFFF, seed >> 32]))
        assert got == want


def test_uniforms_grid_and_range(orc):
    u = orc.sample("uniform", 200000, seed=3)
    assert u.min() > 0.0 and u.max() < 1.0
    k = u * 2 ** 23 - 0.5  # 23-bit grid plus one half
    assert np.array_equal(k, np.round(k))
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)  # exact in FP32
    hist = np.bincount((u * 100).astype(int), minlength=100)
    assert stats.chisquare(hist).pvalue > 1e-3
    w = orc.sample("uniform", 200000, seed=3, wide=True)
    assert w.min() > 0.0 and w.max() < 1.0
    assert stats.kstest(w, "uniform").pvalue > 1e-3


# ---------------------------------------------------------------- cross sections
def _kn_dsigma_dcos(e, c):
    k = e / MEC2
    p = 1.0 / (1.0 + k * (1.0 - c))
    return math.pi * RE * RE * p * p * (p + 1.0 / p - (1.0 - c * c))


@pytest.mark.parametrize("e", [0.001, 0.01, 0.03, 0.1, 0.2, 0.3405, 0.511])
def test_sigma_kn_against_integrated_differential(orc, e):
    val, _ = integrate.quad(lambda c: _kn_dsigma_dcos(e, c), -1.0, 1.0, epsabs=0,
                            epsrel=1e-13, limit=200)
    assert orc.sigma_kn(e) == pytest.approx(val, rel=1e-10, abs=0)


def test_sigma_kn_thomson_limit(orc):
    sig_t = 8.0 * math.pi / 3.0 * RE * RE
    # first-order low-energy expansion: sigma = sigma_T (1 - 2k + ...)
    k = 1e-3 / MEC2
    assert orc.sigma_kn(1e-3) == pytest.approx(sig_t * (1 - 2 * k + 5.2 * k * k), rel=1e-6, abs=0)


def test_cross_section_anchors_and_scaling(orc):
    for zoa in (0.5551, 0.515):
        c = orc.mass_atten(1, 7.4, zoa, 0.030, interp=False)
        pe = orc.mass_atten(2, 7.4, zoa, 0.030, interp=False)
        r = orc.mass_atten(3, 7.4, zoa, 0.030, interp=False)
        assert pe == pytest.approx(c, rel=1e-13, abs=0)       # PE equals Compton at 30 keV, Z 7.4
        assert r == pytest.approx(0.1 * c, rel=1e-13, abs=0)  # Rayleigh is a tenth of it
        assert c == pytest.approx(NA * zoa * orc.sigma_kn(0.030), rel=1e-14, abs=0)
    # per-atom Z^4 and Z^2 laws -> per-gram Z^3 and Z at fixed Z/A
    z1, z2 = 7.4, 12.3
    assert orc.mass_atten(2, z2, 0.5, 0.1, False) / orc.mass_atten(2, z1, 0.5, 0.1, False) == \
        pytest.approx((z2 / z1) ** 3, rel=1e-13, abs=0)
    assert orc.mass_atten(3, z2, 0.5, 0.1, False) / orc.mass_atten(3, z1, 0.5, 0.1, False) == \
        pytest.approx(z2 / z1, rel=1e-13, abs=0)
    # energy laws E^-3, E^-2
    assert orc.mass_atten(2, z1, 0.5, 0.05, False) / orc.mass_atten(2, z1, 0.5, 0.1, False) == \
        pytest.approx(8.0, rel=1e-13, abs=0)
    assert orc.mass_atten(3, z1, 0.5, 0.05, False) / orc.mass_atten(3, z1, 0.5, 0.1, False) == \
        pytest.approx(4.0, rel=1e-13, abs=0)


def test_log_grid_and_interpolation(orc):
    e = np.array([orc.grid_energy(i) for i in range(256)])
    assert e[0] == pytest.approx(1e-3, rel=1e-15, abs=0) and e[-1] == pytest.approx(0.511, rel=1e-14, abs=0)
    assert np.allclose(np.diff(np.log(e)), math.log(511.0) / 255.0, rtol=1e-12, atol=0)
    # nodes reproduced; power laws exact between nodes; KN within 1.1e-5
    for i in (0, 17, 128, 254):
        assert orc.mass_atten(1, 7.4, 0.55, e[i]) == pytest.approx(
            orc.mass_atten(1, 7.4, 0.55, e[i], interp=False), rel=1e-13, abs=0)
    grid = np.exp(np.linspace(math.log(0.0105), math.log(0.5105), 3001))
    err = max(abs(orc.mass_atten(1, 7.4, 0.55, x) / orc.mass_atten(1, 7.4, 0.55, x, False) - 1)
              for x in grid)
    assert err < 1.1e-5
    for p in (2, 3):
        err = max(abs(orc.mass_atten(p, 7.4, 0.55, x) / orc.mass_atten(p, 7.4, 0.55, x, False)
                      - 1) for x in grid[::10])
        assert err < 1e-12


def test_water_attenuation_at_511(orc):
    # total linear attenuation of unit-density water (Z/A 0.5551) at 511 keV,
    # from the integrated KN cross section plus the two power laws
    sig511, _ = integrate.quad(lambda c: _kn_dsigma_dcos(0.511, c), -1, 1, epsrel=1e-13)
    sig30, _ = integrate.quad(lambda c: _kn_dsigma_dcos(0.030, c), -1, 1, epsrel=1e-13)
    ne = NA * 0.5551
    mu = ne * (sig511 + sig30 * (0.030 / 0.511) ** 3 + 0.1 * sig30 * (0.030 / 0.511) ** 2)
    got = sum(orc.mass_atten(p, 7.4, 0.5551, 0.511) for p in (1, 2, 3))
    assert got == pytest.approx(mu, rel=2e-6, abs=0)
    assert 0.0958 < got < 0.0960


# ---------------------------------------------------------------- samplers
def _kn_bin_masses(e, edges):
    tot, _ = integrate.quad(lambda c: _kn_dsigma_dcos(e, c), -1, 1, epsrel=1e-12)
    return np.array([integrate.quad(lambda c: _kn_dsigma_dcos(e, c), a, b, epsrel=1e-12)[0]
                     for a, b in zip(edges[:-1], edges[1:])]) / tot


@pytest.mark.parametrize("kind", ["kahn", "butcher"])
@pytest.mark.parametrize("e", [0.511, 0.2, 0.05])
def test_kn_sampler_chi2(orc, kind, e):
    n = 1_000_000
    s = orc.sample(kind, n, seed=11 + int(e * 1000), e_mev=e, wide=True)
    eps, c = s[:, 0], s[:, 1]
    k = e / MEC2
    # eps and cos are tied by Compton kinematics
    assert np.allclose(c, 1.0 - (1.0 / eps - 1.0) / k, atol=1e-12)
    assert eps.min() >= 1.0 / (1.0 + 2.0 * k) - 1e-15 and eps.max() <= 1.0 + 1e-15
    edges = np.linspace(-1, 1, 101)
    obs = np.histogram(c, bins=edges)[0]
    exp = _kn_bin_masses(e, edges) * n
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, 99) > 1e-3


def test_kn_mean_energy_transfer_511(orc):
    e = 0.511
    tot, _ = integrate.quad(lambda c: _kn_dsigma_dcos(e, c), -1, 1, epsrel=1e-13)
    k = e / MEC2

    def frac(c):
        return 1.0 - 1.0 / (1.0 + k * (1.0 - c))

    mt, _ = integrate.quad(lambda c: frac(c) * _kn_dsigma_dcos(e, c), -1, 1, epsrel=1e-13)
    mt /= tot
    assert mt == pytest.approx(0.344482, abs=2e-6)
    for kind in ("kahn", "butcher"):
        s = orc.sample(kind, 2_000_000, seed=5, e_mev=e, wide=True)
        t = 1.0 - s[:, 0]
        assert abs(t.mean() - mt) < 4 * t.std() / math.sqrt(len(t))


def test_thomson_inverse_and_chi2(orc):
    for u in np.linspace(1e-6, 1 - 1e-6, 41):
        c = orc.thomson_inverse(u)
        assert -1.0 <= c <= 1.0
        assert (c ** 3 + 3 * c + 4) / 8 == pytest.approx(u, abs=1e-12)
    c = orc.sample("thomson", 500000, seed=4)
    edges = np.linspace(-1, 1, 51)
    F = (edges ** 3 + 3 * edges + 4) / 8
    exp = np.diff(F) * len(c)
    obs = np.histogram(c, bins=edges)[0]
    assert stats.chi2.sf(((obs - exp) ** 2 / exp).sum(), 49) > 1e-3


def test_marsaglia_isotropy(orc):
    d = orc.sample("marsaglia", 400000, seed=8)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    n = len(d)
    assert np.all(np.abs(d.mean(axis=0)) < 4 * math.sqrt(1 / 3 / n))
    assert np.all(np.abs((d ** 2).mean(axis=0) - 1 / 3) < 4 * math.sqrt(4 / 45 / n))
    assert abs((d[:, 0] * d[:, 1]).mean()) < 4 * math.sqrt(1 / 15 / n)
    assert stats.kstest(d[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    phi = np.arctan2(d[:, 1], d[:, 0])
    assert stats.kstest(phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3


def test_rotation_keeps_angle_and_is_uniform_in_azimuth(orc):
    rng = np.random.default_rng(0)
    for d0 in ([0, 0, 1], [0, 0, -1], [1, 0, 0], [0.3, -0.5, 0.81],
               [0.0, 0.0044, 0.99999]):
        d0 = np.array(d0, float)
        d0 /= np.linalg.norm(d0)
        cost = 0.37
        outs = np.array([orc.rotate(d0, cost, u) for u in rng.random(4000)])
        assert np.allclose(np.linalg.norm(outs, axis=1), 1.0, atol=1e-14)
        assert np.allclose(outs @ d0, cost, atol=1e-9)
        # azimuthal average of the new direction is cos(theta) * d0
        assert np.allclose(outs.mean(axis=0), cost * d0, atol=0.04)
