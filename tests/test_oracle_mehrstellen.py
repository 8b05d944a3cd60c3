"""Pins of the oracle's fourth-order (Hermitian, Mehrstellen) discretisation.

The paper notes after Eq. 21 that higher-order Hermitian discretisations
could replace the seven-point Laplacian.  The oracle's stencil 1 uses the
19-point Mehrstellen Laplacian A with its right-hand-side operator B, a
four-point central gradient, and diffusion smoothing with step weight
nu <= 1/6.  What fixes each part, with no implementation to compare with:

* A and B are diagonal on Fourier modes (translation invariant, symmetric),
  annihilate (A) or preserve (B) constants, and the pair solves the Poisson
  equation to fourth order: B(k)/A(k) = -1/(k h)^2 (1 + O((k h)^4));
* the converged potential is the exact discrete solution of
  A phi = -(4 pi / h) B q^s (a DFT solve);
* the whole step converges to brute-force Ewald at fourth order in h
  (error ratio ~16 per halving) where the seven-point form converges at
  second order (~4);
* the net long-range force vanishes (antisymmetric gradient, symmetric
  operators).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_31379_amd import inputs


def fourier_mode(n, k, phase=0.3):
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.cos(2 * np.pi * (k[0] * xx + k[1] * yy + k[2] * zz) / n + phase)


def eigenvalue(op, n, k):
    """The factor op applies to a Fourier mode (checked to be a pure factor)."""
    v = fourier_mode(n, k)
    w = op(v)
    lam = (w * v).sum() / (v * v).sum()
    assert np.max(np.abs(w - lam * v)) < 1e-12 * max(1.0, abs(lam)), k
    return lam


def test_operators_are_diagonal_on_fourier_modes_and_fix_constants():
    n = 8
    for k in [(1, 0, 0), (2, 3, 1), (4, 4, 4), (0, 5, 7), (3, 3, 0)]:
        eigenvalue(O.apply_a19, n, k)
        eigenvalue(O.apply_b, n, k)
    c = np.full((n, n, n), 1.7)
    assert np.max(np.abs(O.apply_a19(c))) < 1e-14
    assert np.max(np.abs(O.apply_b(c) - c)) < 1e-14
    # symmetric: <u, A v> = <A u, v>
    rng = np.random.default_rng(3)
    u, v = rng.normal(size=(n, n, n)), rng.normal(size=(n, n, n))
    assert abs((u * O.apply_a19(v)).sum() - (O.apply_a19(u) * v).sum()) < 1e-11
    assert abs((u * O.apply_b(v)).sum() - (O.apply_b(u) * v).sum()) < 1e-11


def test_poisson_solution_is_fourth_order():
    """-(k h)^2 B(k)/A(k) - 1 falls by 16 per halving of k h along an axis, a
    face diagonal and a body diagonal; the seven-point M gives 4."""
    n = 128
    for d in [(1, 0, 0), (1, 1, 0), (1, 1, 1)]:
        err_ho, err_7 = [], []
        for m in (8, 4, 2):
            k = tuple(m * c for c in d)
            kh2 = sum((2 * math.pi * kk / n) ** 2 for kk in k)
            a = eigenvalue(O.apply_a19, n, k)
            b = eigenvalue(O.apply_b, n, k)
            mm = eigenvalue(O.apply_m, n, k)
            err_ho.append(abs(-kh2 * b / a - 1.0))
            err_7.append(abs(-kh2 / mm - 1.0))
        r_ho = np.array(err_ho[:-1]) / np.array(err_ho[1:])
        r_7 = np.array(err_7[:-1]) / np.array(err_7[1:])
        assert np.all((r_ho > 14.0) & (r_ho < 18.0)), (d, err_ho, r_ho)
        assert np.all((r_7 > 3.5) & (r_7 < 4.5)), (d, err_7, r_7)


def exact_phi_ho(qs, h):
    """DFT solution of A phi = -(4 pi / h) B q^s with zero mean, from the
    operators' symbols computed independently of the oracle's stencils."""
    n = qs.shape[0]
    c = np.cos(2 * np.pi * np.arange(n) / n)
    cx, cy, cz = c[None, None, :], c[None, :, None], c[:, None, None]
    a = (4 * (cx + cy + cz) + 4 * (cx * cy + cy * cz + cz * cx) - 24) / 6.0
    b = (2 * (cx + cy + cz) + 6) / 12.0
    a[0, 0, 0] = 1.0
    ph = -4 * np.pi / h * np.fft.fftn(qs) * b / a
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))


def test_converged_potential_is_the_exact_fourth_order_solution():
    s = inputs.random_neutral(40, 12.0, seed=2, dmin=1.0)
    o = O.Oracle(O.make_params(12.0, 0.5, 6.0, 16, 4, tol=1e-12, stencil=1), s.charges)
    o.compute(s.pos)
    pl = o.plan()
    # smoothing step weight nu <= 1/6 with K = ceil(3 sigma_s^2 / h^2)
    assert pl.K == math.ceil(3 * pl.sigma_s2 / pl.h ** 2) and pl.nu_smooth <= 1 / 6 + 1e-15
    qs = o.get_mesh(O.MESH_QS)
    phi = o.get_mesh(O.MESH_PHI)
    ref = exact_phi_ho(qs - qs.mean(), pl.h)
    assert abs(phi.mean()) < 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(phi - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.slow
def test_mesh_step_converges_to_ewald_at_fourth_order():
    s = inputs.random_neutral(16, 12.0, seed=12, dmin=1.5)
    alpha, rc = 0.8, 6.0
    e3, f_ref = O.ewald(s.pos, s.charges, s.box, alpha)
    errs = {0: [], 1: []}
    for st in (0, 1):
        for n in (16, 32, 64):
            o = O.Oracle(O.make_params(12.0, alpha, rc, n, 4, tol=1e-12, stencil=st, max_cycles=64), s.charges)
            f, e, _ = o.compute(s.pos)
            errs[st].append(np.sqrt(((f - f_ref) ** 2).sum() / (f_ref ** 2).sum()))
            o.close()
    r0 = np.array(errs[0][:-1]) / np.array(errs[0][1:])
    r1 = np.array(errs[1][:-1]) / np.array(errs[1][1:])
    assert np.all((r0 > 3.0) & (r0 < 5.5)), (errs[0], r0)
    assert np.all((r1 > 12.0) & (r1 < 20.0)), (errs[1], r1)
    assert errs[1][-1] < 0.05 * errs[0][-1]


def test_net_force_vanishes_fourth_order():
    s = inputs.nacl(128, 25.2 * (128 / 512) ** (1 / 3), 1200.0, seed=21)
    o = O.Oracle(O.make_params(s.box, 0.5, 7.0, 32, 4, tol=1e-11, stencil=1), s.charges)
    f, _, _ = o.compute(s.pos)
    assert np.max(np.abs(f.sum(0))) < 1e-7 * np.max(np.abs(f))


def test_stencil_out_of_range_rejected():
    with pytest.raises(O.OracleError):
        O.plan(O.make_params(10.0, 0.5, 4.0, 16, 4, stencil=2))
