"""GPU: the boundary calls that report what a step computed.

* p3mz_get_potential returns the potential the forces were interpolated from
  (the same mesh as p3mz_get_mesh(ctx, 4));
* p3mz_stats.net_force is the sum of the forces the call wrote (and NaN when
  it wrote none); it vanishes to the solver tolerance (the momentum paragraph
  after Eq. 21);
* p3mz_batch_step is one MD step of every system and returns the forces,
  energies and V-cycle counts of p3mz_batch_md_run;
* p3mz_md_run recomputes the starting forces when the terms change between
  calls instead of kicking with forces of other terms;
* a schedule with no sweeps at all is rejected.
"""
import numpy as np
import pytest

from paper_2606_31379_amd import configs, inputs

from .gpu_util import K_E, GpuCtx, params_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no HIP device")
    return _t


def water_small():
    return inputs.water(300, 31.0 * (300 / 1000) ** (1 / 3), 300.0, seed=77)


@pytest.mark.parametrize("precision", [0, 1])
def test_get_potential_and_net_force(torch, precision):
    s = water_small()
    gp, _ = params_pair(s.box, 0.32, 6.0, 32, 4, tol=1e-8, precision=precision, k_e=K_E, excl_group=3)
    g = GpuCtx(gp, s.charges, torch)
    try:
        for k in range(3):
            f, e, rc = g.compute(s.pos + 0.5 * k * s.vel)
            st = g.stats()
            net = np.array(st.net_force[:])
            ref = f.sum(axis=0)
            scale = np.abs(f).sum()
            assert np.all(np.abs(net - ref) <= 1e-12 * scale), (net, ref)
            # the pair part cancels exactly; the mesh part to the tolerance
            # (FP64) or to the FP32 rounding of the gather (mixed)
            bar = 1e-6 if precision == 0 else 1e-4
            assert np.all(np.abs(net) <= bar * np.abs(f).max()), (net, np.abs(f).max())
            phi = torch.zeros((32,) * 3, dtype=torch.float64, device="cuda")
            g.P.p3mz_get_potential(g.h, phi.data_ptr(), g.stream())
            torch.cuda.synchronize()
            assert np.array_equal(phi.cpu().numpy(), g.get_mesh(4))
            assert abs(phi.cpu().numpy().mean()) < 1e-12 * np.abs(phi.cpu().numpy()).max()
        # no forces written: the net force is unknown
        g.P.p3mz_compute(g.h, g.pos.data_ptr(), None, None, g.stream())
        torch.cuda.synchronize()
        assert np.all(np.isnan(np.array(g.stats().net_force[:])))
    finally:
        g.close()


def _md_terms(P):
    t = P.p3mz_mdterms()
    t.force_to_acc = 1.0 / 103.6427
    t.mv2_to_energy = 103.6427
    t.model, t.bm_a, t.bm_rho = 1, 4000.0, 0.317
    return t


def test_batch_step_equals_batch_md_run(torch):
    from paper_2606_31379_amd import p3maze as P
    reps = [r for r in configs.nacl_batch(64) if r.n_atoms < 2000][:4]
    systems = [inputs.nacl(r.n_atoms, r.box, r.temp_k, r.seed) for r in reps]
    n = [s.n for s in systems]
    q = np.ascontiguousarray(np.concatenate([s.charges for s in systems]))
    prm = [P.make_params(r.box, 0.30, 9.0, r.mesh, 4, tol=1e-8, precision=1, coulomb_k=K_E) for r in reps]
    dev = torch.device("cuda")
    cat = lambda key: torch.from_numpy(np.ascontiguousarray(np.concatenate([getattr(s, key) for s in systems]))).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    terms = _md_terms(P)
    a, b = P.p3mz_batch_create(prm, n, q), P.p3mz_batch_create(prm, n, q)
    try:
        pa, va, ma = cat("pos"), cat("vel"), cat("masses")
        pb, vb, mb = pa.clone(), va.clone(), ma.clone()
        force = torch.zeros_like(pa)
        energies = torch.zeros((len(n), 4), dtype=torch.float64, device=dev)
        cyc_a = torch.zeros(len(n), dtype=torch.int32, device=dev)
        cyc_b = torch.zeros((len(n), 1), dtype=torch.int32, device=dev)
        for _ in range(3):
            P.p3mz_batch_step(a, pa.data_ptr(), va.data_ptr(), ma.data_ptr(), terms, 0.5, force.data_ptr(),
                              energies.data_ptr(), cyc_a.data_ptr(), stream)
            P.p3mz_batch_md_run(b, pb.data_ptr(), vb.data_ptr(), mb.data_ptr(), terms, 0.5, 1, None, cyc_b.data_ptr(),
                                stream)
            torch.cuda.synchronize()
            assert torch.equal(pa, pb) and torch.equal(va, vb)
            assert torch.equal(cyc_a, cyc_b[:, 0])
            for r in range(len(n)):
                st = P.p3mz_batch_get_stats(b, r)
                e = energies[r].cpu().numpy()
                assert (e[0], e[1], e[3]) == (st.e_sr, st.e_lr, st.e_total)
        # the returned force is the one the closing half kick used: one more
        # half kick with it reproduces the velocity update of the next step
        assert torch.isfinite(force).all() and force.abs().max() > 0
    finally:
        P.p3mz_batch_destroy(a)
        P.p3mz_batch_destroy(b)


def test_md_run_recomputes_forces_when_terms_change(torch):
    from paper_2606_31379_amd import p3maze as P
    s = inputs.nacl(256, 25.2 * 0.5 ** (1 / 3), 1200.0, seed=91)
    gp, _ = params_pair(s.box, 0.30, 6.0, 16, 4, tol=1e-8, precision=0, k_e=K_E)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    salt = _md_terms(P)
    none = _md_terms(P)
    none.model = 0
    runs = []
    for first in (None, none):
        h = P.p3mz_create(gp, s.charges)
        try:
            pos = torch.from_numpy(s.pos.copy()).to(dev)
            vel = torch.from_numpy(s.vel.copy()).to(dev)
            mass = torch.from_numpy(s.masses.copy()).to(dev)
            if first is not None:
                # forces of other terms at the same positions, no step taken
                P.p3mz_md_run(h, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), first, 0.5, 0, None, None, stream)
            P.p3mz_md_run(h, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), salt, 0.5, 3, None, None, stream)
            torch.cuda.synchronize()
            runs.append(pos.cpu().numpy())
        finally:
            P.p3mz_destroy(h)
    # same trajectory up to the solver tolerance (the second context has one
    # more potential in its history); kicking with the forces of the other
    # terms would miss the repulsion, moving ions by ~1e-3 A in three steps
    assert np.max(np.abs(runs[0] - runs[1])) < 1e-6


def test_schedule_without_sweeps_rejected(torch):
    from paper_2606_31379_amd import p3maze as P
    with pytest.raises(P.P3MZError) as ei:
        P.p3mz_create(P.make_params(10.0, 0.5, 4.0, 16, 4, nu_pre=0, nu_post=0), np.array([1.0, -1.0]))
    assert ei.value.code == P.P3MZ_ERR_INVALID_ARG
