"""GPU: short-range pair sums over Verlet neighbour lists with a skin against
the plain cell scan on the same inputs -- forces and energies along a
trajectory, the rebuild trigger at half the skin, the fallback for atoms over
the list capacity, the MD pair terms, and argument checks."""
import numpy as np
import pytest

from paper_2606_31379_amd import configs

from .gpu_util import K_E, GpuCtx, params_pair, rel_rms, trajectory

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no HIP device")
    return _t


WORKLOADS = {"nacl": configs.nacl_512, "water-3000": configs.water_3000,
             "water-24000": lambda: configs.water_sweep(0)}


def make_ctx(w, s, torch, precision=0):
    gp, _ = params_pair(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, precision=precision, k_e=K_E,
                        excl_group=w.excl_group)
    return GpuCtx(gp, s.charges, torch)


def check_same(a, b, x, bar=1e-13):
    """Forces and short-range energy of the list context a and the cell-scan
    context b at positions x (the mesh part is the same code on both)."""
    fa, ea, _ = a.compute(x)
    fb, eb, _ = b.compute(x)
    assert rel_rms(fa, fb) < bar, rel_rms(fa, fb)
    assert abs(ea[0] - eb[0]) <= bar * abs(eb[0]), (ea[0], eb[0])
    assert a.stats().cycles == b.stats().cycles


@pytest.mark.parametrize("workload", ["nacl", "water-3000", "water-24000"])
def test_lists_match_cell_scan(torch, workload):
    from paper_2606_31379_amd import p3maze as P
    w = WORKLOADS[workload]()
    s = w.system()
    print(f"neighbour lists vs cell scan: {w.name}", flush=True)
    a, b = make_ctx(w, s, torch), make_ctx(w, s, torch)
    try:
        P.p3mz_set_neighbor_list(b.h, 0.0)
        builds, over, cap = P.p3mz_get_neighbor_stats(a.h)
        assert cap > 0 and cap % 64 == 0 and builds == 0
        assert P.p3mz_get_neighbor_stats(b.h)[2] == 0
        traj = trajectory(s, 6)
        for x in traj:
            check_same(a, b, x)
        builds, over, _ = P.p3mz_get_neighbor_stats(a.h)
        # the first step builds; at 0.5 fs per step the skin lasts for more
        assert 1 <= builds < len(traj) and over == 0, (builds, over)
        assert P.p3mz_get_neighbor_stats(b.h)[0] == 0
    finally:
        a.close()
        b.close()


def test_rebuild_at_half_skin(torch):
    from paper_2606_31379_amd import p3maze as P
    w = configs.water_3000()
    s = w.system()
    a, b = make_ctx(w, s, torch), make_ctx(w, s, torch)
    try:
        skin = 0.9
        P.p3mz_set_neighbor_list(a.h, skin)
        P.p3mz_set_neighbor_list(b.h, 0.0)
        x = s.pos.copy()
        check_same(a, b, x)
        assert P.p3mz_get_neighbor_stats(a.h)[0] == 1
        # one atom 0.45 skin away: still within the list's guarantee
        x1 = x.copy()
        x1[7] += np.array([0.45 * skin, 0.0, 0.0])
        check_same(a, b, x1)
        assert P.p3mz_get_neighbor_stats(a.h)[0] == 1
        # past half the skin (also across the periodic boundary): rebuilt
        x2 = x.copy()
        x2[7] += np.array([0.0, 0.0, 0.55 * skin])
        x2[11] += np.array([w.box, -w.box, 0.0])
        check_same(a, b, x2)
        assert P.p3mz_get_neighbor_stats(a.h)[0] == 2
        # a periodic image alone moves nothing
        x3 = x2.copy()
        x3[100:200] += w.box
        check_same(a, b, x3)
        assert P.p3mz_get_neighbor_stats(a.h)[0] == 2
        # any other configuration: rebuilt on the first step that sees it
        rng = np.random.Generator(np.random.PCG64(5))
        x4 = x2 + rng.normal(scale=0.3, size=x2.shape)
        check_same(a, b, x4)
        assert P.p3mz_get_neighbor_stats(a.h)[0] == 3
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("workload", ["water-3000", "water-24000"])
def test_over_capacity_falls_back_to_cells(torch, workload):
    from paper_2606_31379_amd import p3maze as P
    w = WORKLOADS[workload]()
    s = w.system()
    a, b = make_ctx(w, s, torch), make_ctx(w, s, torch)
    try:
        # 64 entries per atom: far below the ~400 neighbours within r_cut + skin
        P.p3mz_set_neighbor_list(a.h, 0.1 * w.r_cut, 64)
        P.p3mz_set_neighbor_list(b.h, 0.0)
        for x in trajectory(s, 3):
            check_same(a, b, x)
        builds, over, cap = P.p3mz_get_neighbor_stats(a.h)
        assert cap == 64 and builds >= 1 and over >= s.n, (builds, over, cap)
    finally:
        a.close()
        b.close()


def gpu_terms(P, kind):
    from oracle import oracle as O
    t = P.p3mz_mdterms()
    o = O.md_terms(kind)
    for name, _ in P.p3mz_mdterms._fields_:
        setattr(t, name, getattr(o, name))
    return t


@pytest.mark.parametrize("workload,precision", [("nacl", 0), ("water-3000", 0), ("water-3000", 1)])
def test_md_with_lists_matches_cell_scan(torch, workload, precision):
    """The short-range and the non-electrostatic pair terms of MD steps."""
    from paper_2606_31379_amd import p3maze as P
    w = WORKLOADS[workload]()
    s = w.system()
    steps = 8
    dev = torch.device("cuda")
    out = []
    for skin in (0.1 * w.r_cut, 0.0):
        g = make_ctx(w, s, torch, precision)
        try:
            P.p3mz_set_neighbor_list(g.h, skin)
            pos = torch.from_numpy(s.pos.copy()).to(dev)
            vel = torch.from_numpy(s.vel.copy()).to(dev)
            mass = torch.from_numpy(s.masses.copy()).to(dev)
            elog = torch.zeros((steps, 6), dtype=torch.float64, device=dev)
            clog = torch.zeros(steps, dtype=torch.int32, device=dev)
            P.p3mz_md_run(g.h, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), gpu_terms(P, w.kind), w.dt_fs,
                          steps, elog.data_ptr(), clog.data_ptr(), g.stream())
            torch.cuda.synchronize()
            out.append((pos.cpu().numpy(), vel.cpu().numpy(), elog.cpu().numpy(), clog.cpu().numpy(),
                        P.p3mz_get_neighbor_stats(g.h)[0]))
        finally:
            g.close()
    (pa, va, ea, ca, ba), (pb, vb, eb, cb, bb) = out
    assert ba >= 1 and bb == 0
    assert np.array_equal(ca, cb)
    assert np.max(np.abs(pa - pb)) < 1e-10
    assert np.max(np.abs(va - vb)) <= 1e-10 * np.max(np.abs(vb))
    assert np.max(np.abs(ea - eb)) <= 1e-10 * np.max(np.abs(eb))


def test_neighbor_list_arguments(torch):
    from paper_2606_31379_amd import p3maze as P
    w = configs.nacl_512()
    s = w.system()
    g = make_ctx(w, s, torch)
    try:
        for skin, cap in ((-0.1, 0), (w.r_cut * 1.01, 0), (0.5, -1), (float("nan"), 0)):
            with pytest.raises(P.P3MZError) as e:
                P.p3mz_set_neighbor_list(g.h, skin, cap)
            assert e.value.code == P.P3MZ_ERR_INVALID_ARG
        # the context still works with its previous lists
        f, _, rc = g.compute(s.pos)
        assert rc == 0 and np.all(np.isfinite(f))
    finally:
        g.close()
