"""Secondary-electron transport above the electron cutoff -- TEST
INFRASTRUCTURE ONLY.

Section 2.1 tracks electrons down to a 200 keV cutoff and deposits the rest
of their energy on the spot.  Compton electrons of 0.511 MeV photons reach
T_max = E 2k / (1 + 2k) = 340.7 keV (k = E / m c^2 = 1), so some of them
are tracked.  The paper gives no electron model; the reading taken here is
the continuous-slowing-down approximation (CSDA) along a straight line:

* collision stopping power of the Bethe theory for electrons (ICRU Report 37
  form, with the Moller term F^-), no density-effect correction (it vanishes
  for water below about 0.5 MeV and stays under 0.5 % for compact bone at
  these energies), no radiative loss (under 0.5 % of the loss here);
* the electron leaves the Compton vertex along its recoil momentum
  E d_in - E' d_out (momentum conservation) and keeps that direction;
* inside each voxel it loses the energy that its mass path rho * s takes
  off the CSDA range; once the range left above the cutoff is used up in a
  voxel, all of its remaining energy (the part lost on the way down to the
  cutoff and the cutoff energy itself) is deposited in that voxel;
* an electron that leaves the grid takes its energy with it (escaped).

Plain FP64, one electron at a time; scipy's adaptive quadrature and bracketed
root finder serve as the integration and inversion steps.  Only ``tests/``
may import this module; it shares no code with the HIP library.

Pins (tests/test_oracle_electron.py): the stopping power of water against
the published ICRU 37 values, the range between two energies against the
published CSDA ranges, the recoil kinematics against the textbook recoil
angle and the relativistic energy-momentum relation, and the voxel walk
against energy conservation, a brute-force integration of dT/ds, and the
mass-path scaling of the CSDA.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq

MEC2_MEV = 0.51099895
# 2 pi r_e^2 m_e c^2 N_A in MeV cm^2 / mol (CODATA 2018)
HALF_K_MEV_CM2 = 0.1535375
ELECTRON_CUTOFF_MEV = 0.200  # Section 2.1


def stopping_power(t_mev: float, z_over_a: float, i_ev: float) -> float:
    """Mass collision stopping power (MeV cm^2/g) of an electron of kinetic
    energy t_mev in a medium of electron fraction z_over_a (mol/g) and mean
    excitation energy i_ev (eV): the Bethe formula for electrons,
    (K/2)(Z/A)/beta^2 [ln(tau^2 (tau + 2) / (2 (I/mc^2)^2)) + F^-(tau)],
    F^-(tau) = 1 - beta^2 + (tau^2/8 - (2 tau + 1) ln 2) / (tau + 1)^2,
    tau = T / mc^2, without a density-effect term."""
    tau = t_mev / MEC2_MEV
    gamma = tau + 1.0
    beta2 = 1.0 - 1.0 / (gamma * gamma)
    f_minus = 1.0 - beta2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * math.log(2.0)) / (gamma * gamma)
    i_rel = i_ev * 1e-6 / MEC2_MEV
    log_term = math.log(tau * tau * (tau + 2.0) / (2.0 * i_rel * i_rel))
    return HALF_K_MEV_CM2 * z_over_a / beta2 * (log_term + f_minus)


def csda_range(t_lo: float, t_hi: float, z_over_a: float, i_ev: float) -> float:
    """Mass path (g/cm^2) over which an electron slows from t_hi to t_lo:
    the integral of dT / S(T) from t_lo to t_hi."""
    if t_hi <= t_lo:
        return 0.0
    val, _ = quad(lambda t: 1.0 / stopping_power(t, z_over_a, i_ev), t_lo, t_hi,
                  epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def energy_after(t0: float, mass_path: float, z_over_a: float, i_ev: float,
                 t_floor: float = ELECTRON_CUTOFF_MEV) -> float:
    """Kinetic energy after a mass path mass_path (g/cm^2) from t0, for a path
    shorter than the range from t0 down to t_floor: the T1 in (t_floor, t0]
    with csda_range(T1, t0) = mass_path."""
    if mass_path <= 0.0:
        return t0
    full = csda_range(t_floor, t0, z_over_a, i_ev)
    if mass_path >= full:
        raise ValueError("mass path reaches the floor energy")
    return brentq(lambda t1: csda_range(t1, t0, z_over_a, i_ev) - mass_path, t_floor, t0,
                  xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=200)


def compton_electron(e_mev: float, cost: float, d_in, d_out):
    """Kinetic energy and unit direction of the Compton electron of a photon
    of energy e_mev scattered by cos(theta) = cost from direction d_in to
    d_out: T = E - E', E' = E / (1 + k (1 - cos theta)), momentum
    p = E d_in - E' d_out (units MeV/c)."""
    k = e_mev / MEC2_MEV
    e1 = e_mev / (1.0 + k * (1.0 - cost))
    p = e_mev * np.asarray(d_in, dtype=np.float64) - e1 * np.asarray(d_out, dtype=np.float64)
    pn = float(np.linalg.norm(p))
    if pn == 0.0:
        return 0.0, np.asarray(d_in, dtype=np.float64).copy()
    return e_mev - e1, p / pn


def csda_walk(density, material, voxel_cm, z_over_a, i_ev, r, d, t0,
              cutoff: float = ELECTRON_CUTOFF_MEV):
    """Straight-ahead CSDA walk of one electron through a voxel grid.

    density (g/cm^3, > 0) and material (index into z_over_a and i_ev) are
    [nz][ny][nx] arrays; voxel_cm = (dx, dy, dz); the grid's outer corner is
    the origin.  r (cm, inside the grid) is the start, d the unit direction,
    t0 the kinetic energy.  An electron at or below the cutoff deposits t0
    in its voxel.  Returns (deposits, escaped): deposits is a list of
    (flat voxel index, energy) in the order the voxels are crossed, escaped
    the energy carried out of the grid."""
    nz, ny, nx = density.shape
    n = (nx, ny, nz)
    h = tuple(float(x) for x in voxel_cm)
    r = [float(x) for x in r]
    d = [float(x) for x in d]
    iv = [min(max(int(math.floor(r[a] / h[a])), 0), n[a] - 1) for a in range(3)]

    def flat(ix):
        return ix[0] + nx * (ix[1] + ny * ix[2])

    if t0 <= cutoff:
        return [(flat(iv), float(t0))], 0.0
    # Crossing distances along d to the next face of each axis (voxel by
    # voxel traversal of the straight track).
    tnext, tstep, step = [0.0] * 3, [0.0] * 3, [0] * 3
    for a in range(3):
        if d[a] > 0.0:
            step[a], tnext[a], tstep[a] = 1, ((iv[a] + 1) * h[a] - r[a]) / d[a], h[a] / d[a]
        elif d[a] < 0.0:
            step[a], tnext[a], tstep[a] = -1, (iv[a] * h[a] - r[a]) / d[a], -h[a] / d[a]
        else:
            step[a], tnext[a], tstep[a] = 0, math.inf, math.inf
        tnext[a] = max(tnext[a], 0.0)
    deposits = []
    t = float(t0)
    s_cur = 0.0
    while True:
        v = flat(iv)
        m = int(material[iv[2], iv[1], iv[0]])
        rho = float(density[iv[2], iv[1], iv[0]])
        za, ie = float(z_over_a[m]), float(i_ev[m])
        ax = int(np.argmin(tnext))
        seg = tnext[ax] - s_cur
        need = csda_range(cutoff, t, za, ie)
        if rho * seg >= need:
            deposits.append((v, t))
            return deposits, 0.0
        t1 = energy_after(t, rho * seg, za, ie, cutoff)
        deposits.append((v, t - t1))
        t = t1
        s_cur = tnext[ax]
        iv[ax] += step[ax]
        tnext[ax] += tstep[ax]
        if iv[ax] < 0 or iv[ax] >= n[ax]:
            return deposits, t
