"""Pins of the oracle's OVRVO Langevin thermostat: its counter-based
generator against the generator's published known-answer vectors, the
normals' moments, the friction-free limit (plain velocity Verlet), and the
velocity distribution of the strong-friction limit (Maxwell-Boltzmann)."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_31379_amd import configs

KAT = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
K_E = 14.3996454784


def test_philox_known_answers():
    rows = [line.split() for line in open(KAT) if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        assert O.philox4x32_10(w[0:4], w[4:6]) == w[6:10]


def test_normals_moments():
    z = np.array([O.thermo_normals(12345, a, step, half) for a in range(2000) for step in (0, 7, 1 << 33)
                  for half in (0, 1)])
    # 12,000 triples: mean 0 and variance 1 per component (standard errors
    # 0.009 and 0.013), no correlation between the components
    assert np.all(np.abs(z.mean(axis=0)) < 0.04), z.mean(axis=0)
    assert np.all(np.abs(z.var(axis=0) - 1.0) < 0.06), z.var(axis=0)
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 0.04), c
    # fourth moment of a normal: 3
    assert np.all(np.abs((z ** 4).mean(axis=0) - 3.0) < 0.25)
    # distinct counters and keys give distinct numbers
    assert not np.array_equal(O.thermo_normals(1, 5, 3, 0), O.thermo_normals(1, 5, 3, 1))
    assert not np.array_equal(O.thermo_normals(1, 5, 3, 0), O.thermo_normals(2, 5, 3, 0))
    assert not np.array_equal(O.thermo_normals(1, 5, 3, 0), O.thermo_normals(1, 5, 3 + (1 << 32), 0))


def nacl_oracle():
    w = configs.nacl_512()
    s = w.system()
    op = O.make_params(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, predictor=3, coulomb_k=K_E)
    return w, s, O.Oracle(op, s.charges)


def test_zero_friction_is_velocity_verlet():
    w, s, a = nacl_oracle()
    _, _, b = nacl_oracle()
    try:
        b.set_thermostat(0.0, 0.1, 99)
        ra = a.md_run(s.pos, s.vel, s.masses, O.md_terms(w.kind), w.dt_fs, 2)
        rb = b.md_run(s.pos, s.vel, s.masses, O.md_terms(w.kind), w.dt_fs, 2)
        for x, y in zip(ra[:4], rb[:4]):
            assert np.array_equal(x, y)
    finally:
        a.close()
        b.close()


def test_strong_friction_draws_maxwell_boltzmann():
    """With gamma dt / 2 = 40 the last O update forgets the velocities: they
    are sqrt(kT / m') z, so v sqrt(m' / kT) has unit variance and the kinetic
    energy is 3/2 N kT on average."""
    w, s, o = nacl_oracle()
    try:
        t = O.md_terms(w.kind)
        kt = 0.1034
        o.set_thermostat(80.0 / w.dt_fs, kt, 7)
        _, vel, elog, _, _ = o.md_run(s.pos, s.vel, s.masses, t, w.dt_fs, 1)
        u = vel * np.sqrt(s.masses[:, None] * t.mv2_to_energy / kt)
        # 1,536 components: standard error of the variance 0.036
        assert abs(u.var() - 1.0) < 0.12, u.var()
        assert abs(u.mean()) < 0.08
        assert abs(elog[0, 4] / (1.5 * s.n * kt) - 1.0) < 0.12
        # exactly the scaled normals of the step's second half
        z = np.array([O.thermo_normals(7, a, 0, 1) for a in range(s.n)])
        c = math.exp(-40.0)
        assert np.max(np.abs(u - z)) < 1e-12 + 10 * c * np.max(np.abs(u))
    finally:
        o.close()


def test_thermostat_rejects_bad_arguments():
    _, _, o = nacl_oracle()
    try:
        for g, kt in ((-1.0, 0.1), (0.1, -0.1), (float("nan"), 0.1), (0.1, float("inf"))):
            with pytest.raises(O.OracleError):
                o.set_thermostat(g, kt, 0)
    finally:
        o.close()
