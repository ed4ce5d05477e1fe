"""Pins of the oracle's multiple scattering and straggling in brass (the
aperture block's material, Methods B) and through the voxel loop (Methods A
steps in the patient grid), against closed forms that do not use the
oracle's own scattering or straggling tables (no GPU).

* Brass constants: the radiation length from the mixture rule of copper and
  zinc radiation lengths (1/X0 = sum w_i / X0_i) and Z/A from the elements,
  read back through the scattering-power and straggling tables.
* Brass slabs 1-5 mm at 100-200 MeV: exit-angle variance equals the
  Fermi-Eyges A0 of the scattering power (13.6 MeV / pv)^2 / X0 along the CSDA
  path; exit-energy variance equals Bohr's thin-absorber variance (small
  energy loss per slab).
* Pencil beams through the voxel loop (hinge steps voxel by voxel, the end
  point kept in its voxel): exit moments of position, angle and their
  correlation equal Fermi-Eyges A2, A0, A1; the exit-energy variance after a
  thick water slab equals the first-order propagation of Bohr's variance
  through the CSDA relation (each fluctuation at depth z reaches the exit
  scaled by S(E_exit)/S(E(z))), 68 % above the thin-absorber sum there.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2307_01416_amd import inputs as I

MP_C2 = 938.27208816        # MeV, proton mass (CODATA 2018)
ES = 13.6                   # MeV, scattering-power constant (reading R7)
# elemental data: Z, A (g/mol), radiation length (g/cm^2), mean excitation (eV)
CU = (29, 63.546, 12.86, 322.0)
ZN = (30, 65.38, 12.43, 330.0)
W_CU, W_ZN = 0.63, 0.37     # brass by mass
X0_WATER = 36.08
BOHR = 4.0 * math.pi * 6.02214076e23 * (2.8179403262e-13) ** 2 * 0.51099895 ** 2   # MeV^2 cm^2/g per Z/A


def pv(E):
    return E * (E + 2.0 * MP_C2) / (E + MP_C2)


def beta2(E):
    g = 1.0 + E / MP_C2
    return 1.0 - 1.0 / (g * g)


def x0_brass():
    return 1.0 / (W_CU / CU[2] + W_ZN / ZN[2])


def za_brass():
    return W_CU * CU[0] / CU[1] + W_ZN * ZN[0] / ZN[1]


def _quad(f, a, b):
    return integrate.quad(f, a, b, epsrel=1e-10, limit=400)[0]


# ----------------------------------------------------------- brass constants
def test_brass_radiation_length_from_mixture_rule(orc):
    E = orc.table(orc.M_BRASS, "E")
    T = orc.table(orc.M_BRASS, "T")
    x0 = x0_brass()
    assert x0 == pytest.approx(12.6975, rel=1e-5)
    # scattering power T = (E_s / pv)^2 / X0 at every node: X0 read back
    np.testing.assert_allclose(T * (pv(E) / ES) ** 2 * x0, 1.0, rtol=5e-6)
    # and distinct from water's (a swapped material would fail)
    Tw = orc.table(orc.M_WATER, "T")
    np.testing.assert_allclose(T / Tw, X0_WATER / x0, rtol=5e-6)


def test_brass_z_over_a_from_elements(orc):
    E = orc.table(orc.M_BRASS, "E")
    W = orc.table(orc.M_BRASS, "omega2")
    b2 = beta2(E)
    za = W / (BOHR * (1.0 - 0.5 * b2) / (1.0 - b2))
    np.testing.assert_allclose(za, za_brass(), rtol=1e-6)
    # mean excitation energy by Bragg additivity of ln I weighted by electrons
    lnI = (W_CU * CU[0] / CU[1] * math.log(CU[3]) + W_ZN * ZN[0] / ZN[1] * math.log(ZN[3])) / za_brass()
    assert math.exp(lnI) == pytest.approx(324.947, rel=1e-5)
    # the brass stopping power's I enters through the Bethe log: S_brass/S_water at
    # the same E differs from the Z/A ratio by the log term of the two I values
    S_b = orc.stopping_power(orc.M_BRASS, 150.0)
    S_w = orc.stopping_power(orc.M_WATER, 150.0)
    g = 1.0 + 150.0 / MP_C2
    bg2 = g * g - 1.0
    me = 0.51099895
    tmax = 2 * me * bg2 / (1 + 2 * g * me / MP_C2 + (me / MP_C2) ** 2)
    L = lambda I_ev: 0.5 * math.log(2 * me * bg2 * tmax / (I_ev * 1e-6) ** 2) - beta2(150.0)
    assert S_b / S_w == pytest.approx(za_brass() * L(math.exp(lnI)) / (0.55508 * L(75.0)), rel=1e-4)


# ------------------------------------------------------------- brass slabs
BRASS_RHO = 8.5
SLABS = [(1.0, 100.0), (1.0, 150.0), (1.0, 200.0), (3.0, 100.0), (3.0, 150.0), (3.0, 200.0),
         (5.0, 100.0), (5.0, 150.0), (5.0, 200.0)]


def _brass_energy_along(orc, e0):
    R0 = orc.csda_range(orc.M_BRASS, e0)
    return lambda z: float(orc.energy_of_range(orc.M_BRASS, R0 - BRASS_RHO * z / 10.0))


@pytest.mark.parametrize("L,e0", SLABS)
def test_brass_slab_angle_variance_fermi_eyges(orc, L, e0):
    n = 100_000
    out = orc.slab_exit(orc.M_BRASS, BRASS_RHO, L, e0, physics=2, n=n, seed=4001 + int(10 * L + e0))
    assert np.all(out[:, 0] == 1)
    Ez = _brass_energy_along(orc, e0)
    x0 = x0_brass()
    a0 = _quad(lambda z: (ES / pv(Ez(z))) ** 2 / x0 * BRASS_RHO / 10.0, 0.0, L)
    # both projected components (u and v), 2n normal samples of variance a0;
    # the 1-2 hinge steps evaluate T at each step's mean energy (midpoint rule,
    # < 0.1 % here)
    var = 0.5 * (np.mean(out[:, 4] ** 2) + np.mean(out[:, 5] ** 2))
    assert var == pytest.approx(a0, rel=3.0 * math.sqrt(1.0 / n) + 1e-3)


@pytest.mark.parametrize("L,e0", [se for se in SLABS if se != (5.0, 100.0)])
def test_brass_slab_energy_variance_bohr(orc, L, e0):
    """Bohr's thin-absorber variance int rho omega^2(E(z)) dz, with omega^2 from
    the elements' Z/A (not the oracle's table), where one condensed-history
    step spans the slab (energy loss <= 15 %)."""
    n = 200_000
    out = orc.slab_exit(orc.M_BRASS, BRASS_RHO, L, e0, physics=1, n=n, seed=5003 + int(10 * L + e0))
    Ez = _brass_energy_along(orc, e0)
    assert (e0 - Ez(L)) / e0 <= 0.15
    w2 = lambda E: BOHR * za_brass() * (1.0 - 0.5 * beta2(E)) / (1.0 - beta2(E))
    ref = _quad(lambda z: w2(Ez(z)) * BRASS_RHO / 10.0, 0.0, L)
    assert np.var(out[:, 1]) == pytest.approx(ref, rel=3.0 * math.sqrt(2.0 / n) + 1e-3)
    # the mean exit energy is the CSDA energy (straggling is unbiased)
    assert np.mean(out[:, 1]) == pytest.approx(Ez(L), abs=4.0 * math.sqrt(ref / n))


# --------------------------------------------- pencil beams through voxels
def _pencil(beam_axis: str, physics: int, e0: float = 150.0):
    """Zero-width pencil beam through 100 mm of water, on a voxel column's
    centre line; beam along +z on 1 mm voxels, or along -x (gantry 90) on
    1 x 1 x 2 mm voxels."""
    spots = I.make_spots([(0.0, 0.0)], e0, 0.0, 10)
    if beam_axis == "z":
        g = I.water_geometry((60, 60, 100), (1.0, 1.0, 1.0))
        beam = I.beam_along_z((30.5, 30.5, 0.0))
        centre, lat, depth_axis, exit_face = (30.5, 30.5), (0, 1), 2, 100.0
    else:
        g = I.water_geometry((100, 60, 30), (1.0, 1.0, 2.0))
        beam = I.beam_coplanar((100.0, 30.5, 31.0), 90.0)
        centre, lat, depth_axis, exit_face = (30.5, 31.0), (1, 2), 0, 0.0
    c = I.Case("pencil", g, [I.Field(beam, spots)], [I.Scenario()], seed=3, physics=physics)
    return c, centre, lat, depth_axis, exit_face


def _water_energy_along(orc, e0):
    R0 = orc.csda_range(orc.M_WATER, e0)
    return lambda z: float(orc.energy_of_range(orc.M_WATER, R0 - z / 10.0))


@pytest.mark.parametrize("axis", ["z", "x"])
def test_pencil_beam_fermi_eyges_moments_through_voxels(orc, axis):
    n = 200_000
    L, e0 = 100.0, 150.0
    c, centre, lat, dax, face = _pencil(axis, physics=2, e0=e0)
    out = orc.patient_exit(c, 0, n, seed=17 if axis == "z" else 19)
    assert np.all(out[:, 0] == 1) and np.all(out[:, 2 + dax] == face)
    Ez = _water_energy_along(orc, e0)
    T = lambda z: (ES / pv(Ez(z))) ** 2 / X0_WATER / 10.0     # rad^2 per mm of water
    A0 = _quad(T, 0.0, L)
    A1 = _quad(lambda z: T(z) * (L - z), 0.0, L)
    A2 = _quad(lambda z: T(z) * (L - z) ** 2, 0.0, L)
    tol = 3.0 * math.sqrt(2.0 / n) + 2e-3
    for j, k in enumerate(lat):
        x = out[:, 2 + k] - centre[j]
        u = out[:, 5 + k]
        assert np.mean(u * u) == pytest.approx(A0, rel=tol)
        assert np.mean(x * x) == pytest.approx(A2, rel=tol)
        # <x u> = A1: relative error of a product moment of correlated normals
        # is sqrt((1 + r^2)/n)/r with r^2 = A1^2/(A0 A2) = 3/4 for a uniform T
        r = A1 / math.sqrt(A0 * A2)
        assert np.mean(x * u) == pytest.approx(A1, rel=3.0 * math.sqrt((1 + r * r) / n) / r + 2e-3)
        # no systematic drift of the centre line (the end-point clamp is symmetric)
        assert abs(np.mean(x)) <= 4.0 * math.sqrt(A2 / n)


def test_straggling_propagates_through_voxel_steps(orc):
    """100 mm of water as 100 voxel steps: the exit-energy variance is Bohr's
    variance propagated to the exit, int omega^2(E(z)) (S(E_L)/S(E(z)))^2 dz
    (68 % above the thin-absorber sum here).  With the point stopping power
    the tolerance carries the CSDA interpolant's secant slopes (within 1 % of
    S over a 2.2 % node interval, squared); with the interpolant's own slopes
    (the range table, pinned to the quadrature of 1/S) only the statistics."""
    n = 1_000_000
    L, e0 = 100.0, 150.0
    c, _, _, _, _ = _pencil("z", physics=1, e0=e0)
    out = orc.patient_exit(c, 0, n, seed=23)
    Ez = _water_energy_along(orc, e0)
    EL = Ez(L)
    w2 = lambda E: BOHR * 0.55508 * (1.0 - 0.5 * beta2(E)) / (1.0 - beta2(E))
    S = lambda E: float(orc.stopping_power(orc.M_WATER, E))
    En, Rn = orc.table(orc.M_WATER, "E"), orc.table(orc.M_WATER, "R")

    def S_seg(E):
        i = int(np.searchsorted(En, E)) - 1
        return (En[i + 1] - En[i]) / (Rn[i + 1] - Rn[i])

    zm = (np.arange(4000) + 0.5) * (L / 4000)
    Ev = np.array([Ez(z) for z in zm])
    dz = L / 4000 / 10.0                      # cm of water per sample
    thin = sum(w2(e) for e in Ev) * dz
    prop = sum(w2(e) * (S(EL) / S(e)) ** 2 for e in Ev) * dz
    prop_seg = sum(w2(e) * (S_seg(EL) / S_seg(e)) ** 2 for e in Ev) * dz
    v = np.var(out[:, 1])
    tol = 3.0 * math.sqrt(2.0 / n)
    assert v == pytest.approx(prop, rel=tol + 0.02)
    assert v == pytest.approx(prop_seg, rel=tol + 2e-3)
    assert v / thin > 1.5                     # the propagation, not the thin sum
