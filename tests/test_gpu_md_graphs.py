"""GPU: the MD driver against the oracle's velocity-Verlet loop, graph replay
against direct launches, and the kernel timing entry points."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_31379_amd import configs

from .gpu_util import K_E, GpuCtx, params_pair, trajectory

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no HIP device")
    return _t


def gpu_terms(P, kind):
    t = P.p3mz_mdterms()
    o = O.md_terms(kind)
    for name, _ in P.p3mz_mdterms._fields_:
        setattr(t, name, getattr(o, name))
    return t


@pytest.mark.parametrize("workload,precision", [("nacl", 0), ("water", 0), ("water", 1)])
def test_md_run_matches_oracle(torch, workload, precision):
    from paper_2606_31379_amd import p3maze as P
    w = configs.nacl_512() if workload == "nacl" else configs.water_3000()
    s = w.system()
    steps = 8
    gp, op = params_pair(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, precision=precision, k_e=K_E,
                         predictor=3, excl_group=w.excl_group)
    o = O.Oracle(op, s.charges)
    po, vo, elog_o, clog_o, _ = o.md_run(s.pos, s.vel, s.masses, O.md_terms(w.kind), w.dt_fs, steps)
    g = GpuCtx(gp, s.charges, torch)
    try:
        dev = torch.device("cuda")
        pos = torch.from_numpy(s.pos.copy()).to(dev)
        vel = torch.from_numpy(s.vel.copy()).to(dev)
        mass = torch.from_numpy(s.masses.copy()).to(dev)
        elog = torch.zeros((steps, 6), dtype=torch.float64, device=dev)
        clog = torch.zeros(steps, dtype=torch.int32, device=dev)
        # two calls: the driver keeps its forces and history between calls
        half = steps // 2
        for k0, k1 in ((0, half), (half, steps)):
            P.p3mz_md_run(g.h, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), gpu_terms(P, w.kind), w.dt_fs,
                          k1 - k0, elog[k0].data_ptr(), clog[k0].data_ptr(), g.stream())
        torch.cuda.synchronize()
        pg, vg = pos.cpu().numpy(), vel.cpu().numpy()
        eg, cg = elog.cpu().numpy(), clog.cpu().numpy()
        assert np.array_equal(cg, clog_o), (cg, clog_o)
        bar = 1e-10 if precision == 0 else 1e-6
        assert np.max(np.abs(pg - po)) < bar * 10, np.max(np.abs(pg - po))
        assert np.max(np.abs(vg - vo)) <= bar * np.max(np.abs(vo)) * 10
        assert np.max(np.abs(eg - elog_o)) <= bar * np.max(np.abs(elog_o)) * 10
    finally:
        g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_equals_direct_launches(torch, precision):
    from paper_2606_31379_amd import p3maze as P
    w = configs.water_3000()
    s = w.system()
    gp, _ = params_pair(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, precision=precision, k_e=K_E,
                        excl_group=3)
    traj = trajectory(s, 6)
    runs = []
    for graphs in (True, False):
        g = GpuCtx(gp, s.charges, torch)
        try:
            P.p3mz_set_graphs(g.h, graphs)
            out = []
            for x in traj:
                f, e, _ = g.compute(x)
                phi = g.get_mesh(4)          # eager work between the replays
                out.append((f, e, phi, g.stats().cycles))
            runs.append(out)
        finally:
            g.close()
    for a, b in zip(*runs):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert a[3] == b[3]


def test_kernel_timers(torch):
    from paper_2606_31379_amd import p3maze as P
    w = configs.water_3000()
    s = w.system()
    gp, _ = params_pair(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, precision=1, k_e=K_E, excl_group=3)
    g = GpuCtx(gp, s.charges, torch)
    try:
        traj = trajectory(s, 3)
        P.p3mz_set_timing(g.h, True)
        # the 64^3 level runs its legs fused (one launch per leg)
        P.p3mz_set_kernel_timer(g.h, P.KERNELS["fused_up"])
        for x in traj:
            g.compute(x)
        ms, n, b = P.p3mz_get_kernel_timer(g.h)
        assert n > 0 and ms > 0 and math.isclose(b / n, 2.625 * 4 * 64 ** 3)
        P.p3mz_set_kernel_timer(g.h, P.KERNELS["halfsweep"])
        g.compute(traj[-1])
        assert P.p3mz_get_kernel_timer(g.h)[1] == 0
        st = g.stats()
        # the kernel timer forces direct launches, so the sub-stages are timed too
        assert st.graphs == 0 and st.ms_mesh > 0 and st.ms_short_range > 0
        assert st.ms_spread > 0 and st.ms_solve > 0 and st.ms_gather > 0
        assert abs(st.ms_spread + st.ms_solve + st.ms_gather - st.ms_mesh) < 1e-3 * st.ms_mesh + 1e-3
        P.p3mz_set_kernel_timer(g.h, -1)
        for name in ("halfsweep", "sweep0", "restrict", "prolong", "tail", "smooth", "fused_down", "fused_up"):
            ms, b = P.p3mz_kernel_bench(g.h, P.KERNELS[name], 5, g.stream())
            assert ms > 0 and b > 0, name
        with pytest.raises(P.P3MZError):
            P.p3mz_kernel_bench(g.h, P.KERNELS["sr"], 1, g.stream())
        # timing and the bursts leave the step itself unchanged; graphs again
        f1, _, _ = g.compute(traj[-1])
        assert np.all(np.isfinite(f1))
        f1, _, _ = g.compute(traj[-1])
        st = g.stats()
        assert st.graphs == 1 and st.ms_mesh > 0 and st.ms_spread == -1.0
    finally:
        g.close()
