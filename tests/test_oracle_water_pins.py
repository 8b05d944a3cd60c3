"""Pins of the oracle's water terms and of its exclusion correction.

Both parts are checked against facts that do not come from the oracle's own
formulas:

* the flexible three-site water model (Supporting Information, table of
  flexible-water parameters: harmonic O-H bonds, harmonic H-O-H angle, O-O
  Lennard-Jones) by closed-form energies of hand-built geometries, the
  geometric size and direction of the bond and angle forces, the
  Lennard-Jones minimum at 2^(1/6) sigma, and central differences of the
  energy;
* the excluded-pair term of the short-range sum (the mesh carries every pair,
  so an excluded pair must lose its smooth part -k_e Q_i Q_j erf(alpha r)/r,
  Eqs. 5-7 and 20) by convergence of the whole step, at second order in h, to
  the brute-force Ewald sum minus the bare Coulomb interaction of the
  excluded pairs.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_31379_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
KCAL_MOL_EV = 0.0433641


def gold(key):
    with open(os.path.join(HERE, "golden", "paper_values.json")) as fh:
        return json.load(fh)[key]["value"]


def water_terms():
    t = O.md_terms("water")
    # the parameters the oracle uses are the paper's table values
    assert t.k_bond == pytest.approx(gold("water_kb_kcal_mol_A2") * KCAL_MOL_EV, rel=1e-15)
    assert t.k_angle == pytest.approx(gold("water_ka_kcal_mol_rad2") * KCAL_MOL_EV, rel=1e-15)
    assert t.r0 == pytest.approx(gold("water_r0_A"), rel=1e-15)
    assert t.theta0 == pytest.approx(math.radians(gold("water_theta0_deg")), rel=1e-15)
    assert t.lj_eps == pytest.approx(gold("water_lj_eps_kcal_mol") * KCAL_MOL_EV, rel=1e-15)
    assert t.lj_sigma == pytest.approx(gold("water_lj_sigma_A"), rel=1e-15)
    return t


def molecule(origin, r1, r2, theta, frame=np.eye(3)):
    """O at origin, H1 at r1 along the frame's first axis, H2 at r2 in the
    frame's first-second plane at angle theta from H1."""
    e1, e2 = frame[0], frame[1]
    o = np.asarray(origin, dtype=float)
    return np.array([o, o + r1 * e1, o + r2 * (math.cos(theta) * e1 + math.sin(theta) * e2)])


def rotation(seed):
    q = np.random.default_rng(seed).standard_normal(4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


BOX, RC = 30.0, 9.0


@pytest.mark.parametrize("r1,r2,dtheta_deg", [(1.05, 0.97, 0.0), (1.012, 1.012, 7.5), (0.93, 1.08, -11.0)])
def test_single_molecule_energy_closed_form(r1, r2, dtheta_deg):
    t = water_terms()
    theta = t.theta0 + math.radians(dtheta_deg)
    pos = molecule([3.1, 4.2, 5.3], r1, r2, theta, rotation(3))
    f, e = O.nonelectrostatic(t, pos, BOX, RC)
    ref = 0.5 * t.k_bond * ((r1 - t.r0) ** 2 + (r2 - t.r0) ** 2) + 0.5 * t.k_angle * (theta - t.theta0) ** 2
    assert e == pytest.approx(ref, rel=1e-12, abs=1e-15)
    # internal forces: no net force and no net torque about the O atom
    assert np.max(np.abs(f.sum(0))) < 1e-12
    torque = np.cross(pos[1] - pos[0], f[1]) + np.cross(pos[2] - pos[0], f[2])
    assert np.max(np.abs(torque)) < 1e-12


def test_bond_force_is_along_the_bond():
    """At the equilibrium angle only the bonds act: the force on each H is
    -k_b (r - r0) along its O-H unit vector."""
    t = water_terms()
    frame = rotation(11)
    pos = molecule([10.0, 11.0, 12.0], 1.09, 0.95, t.theta0, frame)
    f, _ = O.nonelectrostatic(t, pos, BOX, RC)
    for h, r in ((1, 1.09), (2, 0.95)):
        u = (pos[h] - pos[0]) / r
        assert np.allclose(f[h], -t.k_bond * (r - t.r0) * u, rtol=1e-12, atol=1e-13)


def test_angle_force_is_tangential_with_size_k_dtheta_over_r():
    """With both bonds at r0 only the angle acts: the force on each H lies in
    the molecular plane, perpendicular to its bond, of size k_a |theta -
    theta0| / r0, turning the H towards the equilibrium angle."""
    t = water_terms()
    frame = rotation(12)
    for dth in (math.radians(9.0), math.radians(-6.0)):
        theta = t.theta0 + dth
        pos = molecule([5.0, 6.0, 7.0], t.r0, t.r0, theta, frame)
        f, _ = O.nonelectrostatic(t, pos, BOX, RC)
        size = t.k_angle * abs(dth) / t.r0
        b1, b2 = pos[1] - pos[0], pos[2] - pos[0]
        for h, own, other in ((1, b1, b2), (2, b2, b1)):
            assert abs(np.dot(f[h], own)) < 1e-11
            assert abs(np.dot(f[h], np.cross(b1, b2))) < 1e-11
            assert np.linalg.norm(f[h]) == pytest.approx(size, rel=1e-10)
            # an opened angle (dth > 0) pushes each H towards the other bond
            assert np.sign(np.dot(f[h], other)) == np.sign(dth)


def test_lennard_jones_minimum_and_zero_crossing():
    """Two molecules at their equilibrium geometry: the only force is the O-O
    Lennard-Jones one, zero at r = 2^(1/6) sigma with energy -eps - shift, and
    24 eps / sigma (repulsive) at r = sigma with energy -shift, where the
    shift makes the potential vanish at the cutoff."""
    t = water_terms()
    eps, sig = t.lj_eps, t.lj_sigma
    shift = 4 * eps * ((sig / RC) ** 12 - (sig / RC) ** 6)
    ex = np.array([1.0, 0.0, 0.0])
    for r, e_ref, f_ref in ((2 ** (1 / 6) * sig, -eps - shift, 0.0), (sig, -shift, 24 * eps / sig)):
        a = molecule([8.0, 8.0, 8.0], t.r0, t.r0, t.theta0, rotation(5))
        b = molecule(a[0] + r * ex, t.r0, t.r0, t.theta0, rotation(6))
        pos = np.concatenate([a, b])
        f, e = O.nonelectrostatic(t, pos, BOX, RC)
        assert e == pytest.approx(e_ref, rel=1e-12, abs=1e-16)
        assert np.allclose(f[0], -f_ref * ex, atol=1e-12)
        assert np.allclose(f[3], f_ref * ex, atol=1e-12)
        assert np.max(np.abs(f[[1, 2, 4, 5]])) < 1e-12
    # beyond the cutoff nothing acts
    a = molecule([2.0, 2.0, 2.0], t.r0, t.r0, t.theta0)
    b = molecule(a[0] + (RC + 0.01) * ex, t.r0, t.r0, t.theta0)
    f, e = O.nonelectrostatic(t, np.concatenate([a, b]), BOX, RC)
    assert abs(e) < 1e-20 and np.max(np.abs(f)) < 1e-12


def test_water_forces_are_minus_the_energy_gradient():
    """Displaced molecules in a small periodic box (bonds, angles and O-O
    pairs inside the cutoff, some across the box faces): central differences
    of the total energy give the forces."""
    t = water_terms()
    box = 9.5
    s = inputs.water(10, box, 300.0, seed=41, r_oh=1.0, angle_deg=104.0)
    rng = np.random.default_rng(2)
    pos = s.pos + rng.normal(scale=0.05, size=s.pos.shape)
    f, _ = O.nonelectrostatic(t, pos, box, 4.7)
    assert np.max(np.abs(f.sum(0))) < 1e-10
    d = 1e-5
    for i in range(0, 30, 2):
        for k in range(3):
            pp = pos.copy(); pp[i, k] += d
            pm = pos.copy(); pm[i, k] -= d
            g = (O.nonelectrostatic(t, pp, box, 4.7)[1] - O.nonelectrostatic(t, pm, box, 4.7)[1]) / (2 * d)
            assert abs(-g - f[i, k]) < 1e-6 * max(1.0, abs(f[i, k])), (i, k, -g, f[i, k])


# ---------------------------------------------------------------------------
# Exclusion correction against Ewald minus the bare Coulomb of excluded pairs
# ---------------------------------------------------------------------------
def bare_coulomb_of_groups(pos, q, box, g):
    """Energy and forces of the direct (minimum-image) Coulomb interaction of
    every pair inside one group of g consecutive atoms."""
    e = 0.0
    f = np.zeros_like(pos)
    for a in range(0, pos.shape[0], g):
        for i in range(a, a + g):
            for j in range(i + 1, a + g):
                d = pos[i] - pos[j]
                d -= box * np.round(d / box)
                r = np.linalg.norm(d)
                e += q[i] * q[j] / r
                f[i] += q[i] * q[j] * d / r ** 3
                f[j] -= q[i] * q[j] * d / r ** 3
    return e, f


@pytest.mark.slow
def test_exclusion_correction_converges_to_ewald_minus_bare_coulomb():
    """30 molecules at about liquid density; the short-range tail beyond the
    cutoff (erfc(3) ~ 2e-5) stays below the mesh error at 128^3."""
    box, alpha, rc = 10.0, 0.6, 5.0
    s = inputs.water(30, box, 300.0, seed=43)
    e3, f_ew = O.ewald(s.pos, s.charges, box, alpha)
    e_bare, f_bare = bare_coulomb_of_groups(s.pos, s.charges, box, 3)
    e_ref, f_ref = e3.sum() - e_bare, f_ew - f_bare
    errs_f, errs_e = [], []
    for n in (32, 64, 128):
        o = O.Oracle(O.make_params(box, alpha, rc, n, 4, tol=1e-12, excl_group=3), s.charges)
        f, e, st = o.compute(s.pos)
        assert st == 0
        errs_f.append(np.sqrt(((f - f_ref) ** 2).sum() / (f_ref ** 2).sum()))
        errs_e.append(abs(e[3] - e_ref))
        o.close()
    ratios_f = np.array(errs_f[:-1]) / np.array(errs_f[1:])
    ratios_e = np.array(errs_e[:-1]) / np.array(errs_e[1:])
    assert errs_f[-1] < 2e-3, (errs_f, ratios_f)
    assert np.all((ratios_f > 3.3) & (ratios_f < 4.7)), (errs_f, ratios_f)
    assert 3.0 < ratios_e[-1] < 5.0, (errs_e, ratios_e)
    # a sign or factor error in the correction would leave an offset of the
    # order of the excluded pairs' bare Coulomb energy, far above the error
    assert abs(e_bare) > 1e4 * errs_e[-1], (e_bare, errs_e)
