"""GPU: batched replicas.  Every system of a batch must give bitwise the same
forces, energies, potentials and V-cycle counts as the same system run alone
in its own context (each system runs the single-system algorithm; the batch
only merges the launches), for mesh steps along a trajectory and for MD runs,
in FP64 and mixed mode, with graphs and with direct launches.  One replica is
also checked against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_31379_amd import configs

from .gpu_util import K_E, rel_rms

pytestmark = pytest.mark.gpu

# a mix of the replica recipe: meshes 16^3, 32^3 and 64^3, ragged atom counts
PICK = [0, 1, 2, 5, 9]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no HIP device")
    return _t


def replicas(pick, max_atoms=6000):
    reps = configs.nacl_batch(64)
    small = sorted(range(64), key=lambda i: reps[i].n_atoms)
    # keep the test fast: the smallest systems of each mesh size present
    chosen, seen = [], {}
    for i in small:
        r = reps[i]
        if r.n_atoms > max_atoms:
            continue
        if seen.get(r.mesh, 0) < 2:
            chosen.append(r)
            seen[r.mesh] = seen.get(r.mesh, 0) + 1
    return chosen[: len(pick)]


def sys_params(P, r, precision, **kw):
    return P.make_params(r.box, 0.30, 9.0, r.mesh, 4, tol=1e-8, precision=precision, coulomb_k=K_E, **kw)


def build(torch, precision, reps=None):
    from paper_2606_31379_amd import inputs
    reps = reps or replicas(PICK)
    systems = [inputs.nacl(r.n_atoms, r.box, r.temp_k, r.seed) for r in reps]
    return reps, systems


def packed(arrs):
    return np.ascontiguousarray(np.concatenate(arrs, axis=0))


def test_replica_mix():
    reps = replicas(PICK)
    assert len(reps) == 5 and {r.mesh for r in reps} == {16, 32, 64}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("graphs", [True, False])
def test_batch_compute_equals_single(torch, precision, graphs):
    from paper_2606_31379_amd import p3maze as P
    reps, systems = build(torch, precision)
    dev = torch.device("cuda")
    n = [s.n for s in systems]
    q = packed([s.charges for s in systems])
    b = P.p3mz_batch_create([sys_params(P, r, precision) for r in reps], n, q)
    singles = [P.p3mz_create(sys_params(P, r, precision), s.charges) for r, s in zip(reps, systems)]
    for h in singles:
        # batched systems scan the cells for their pairs: so does the reference
        P.p3mz_set_neighbor_list(h, 0.0)
    stream = torch.cuda.current_stream().cuda_stream
    try:
        P.p3mz_batch_set_graphs(b, graphs)
        pos = torch.zeros((sum(n), 3), dtype=torch.float64, device=dev)
        frc = torch.zeros_like(pos)
        en = torch.zeros((len(n), 4), dtype=torch.float64, device=dev)
        spos = [torch.zeros((k, 3), dtype=torch.float64, device=dev) for k in n]
        sfrc = [torch.zeros_like(x) for x in spos]
        sen = [torch.zeros(4, dtype=torch.float64, device=dev) for _ in n]
        for step in range(5):
            xs = [s.pos + step * 0.5 * s.vel for s in systems]
            pos.copy_(torch.from_numpy(packed(xs)))
            P.p3mz_batch_compute(b, pos.data_ptr(), frc.data_ptr(), en.data_ptr(), stream)
            for i, x in enumerate(xs):
                spos[i].copy_(torch.from_numpy(np.ascontiguousarray(x)))
                P.p3mz_compute(singles[i], spos[i].data_ptr(), sfrc[i].data_ptr(), sen[i].data_ptr(), stream)
            torch.cuda.synchronize()
            fb, eb = frc.cpu().numpy(), en.cpu().numpy()
            off = 0
            for i in range(len(n)):
                fs = sfrc[i].cpu().numpy()
                assert np.array_equal(fb[off:off + n[i]], fs), (step, i)
                assert np.array_equal(eb[i], sen[i].cpu().numpy()), (step, i)
                sb, ss = P.p3mz_batch_get_stats(b, i), P.p3mz_get_stats(singles[i])
                assert sb.cycles == ss.cycles and sb.cold == ss.cold and sb.m_eff == ss.m_eff, (step, i)
                assert list(sb.res_hist)[: sb.cycles + 1] == list(ss.res_hist)[: ss.cycles + 1]
                off += n[i]
        if graphs:
            assert P.p3mz_batch_get_timing(b)[2] == 1
    finally:
        P.p3mz_batch_destroy(b)
        for h in singles:
            P.p3mz_destroy(h)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_md_equals_single(torch, precision):
    from paper_2606_31379_amd import p3maze as P
    from .test_gpu_md_graphs import gpu_terms
    reps, systems = build(torch, precision)
    dev = torch.device("cuda")
    n = [s.n for s in systems]
    steps = 6
    b = P.p3mz_batch_create([sys_params(P, r, precision) for r in reps], n, packed([s.charges for s in systems]))
    stream = torch.cuda.current_stream().cuda_stream
    terms = gpu_terms(P, "nacl")
    try:
        pos = torch.from_numpy(packed([s.pos for s in systems])).to(dev)
        vel = torch.from_numpy(packed([s.vel for s in systems])).to(dev)
        mass = torch.from_numpy(packed([s.masses for s in systems])).to(dev)
        elog = torch.zeros((len(n), steps, 6), dtype=torch.float64, device=dev)
        clog = torch.zeros((len(n), steps), dtype=torch.int32, device=dev)
        P.p3mz_batch_md_run(b, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), terms, 0.5, steps,
                            elog.data_ptr(), clog.data_ptr(), stream)
        torch.cuda.synchronize()
        pb, vb, eb, cb = pos.cpu().numpy(), vel.cpu().numpy(), elog.cpu().numpy(), clog.cpu().numpy()
        off = 0
        for i, (r, s) in enumerate(zip(reps, systems)):
            h = P.p3mz_create(sys_params(P, r, precision), s.charges)
            try:
                P.p3mz_set_neighbor_list(h, 0.0)
                p1 = torch.from_numpy(s.pos.copy()).to(dev)
                v1 = torch.from_numpy(s.vel.copy()).to(dev)
                m1 = torch.from_numpy(s.masses.copy()).to(dev)
                e1 = torch.zeros((steps, 6), dtype=torch.float64, device=dev)
                c1 = torch.zeros(steps, dtype=torch.int32, device=dev)
                P.p3mz_md_run(h, p1.data_ptr(), v1.data_ptr(), m1.data_ptr(), terms, 0.5, steps, e1.data_ptr(),
                              c1.data_ptr(), stream)
                torch.cuda.synchronize()
                assert np.array_equal(pb[off:off + s.n], p1.cpu().numpy()), i
                assert np.array_equal(vb[off:off + s.n], v1.cpu().numpy()), i
                assert np.array_equal(eb[i], e1.cpu().numpy()), i
                assert np.array_equal(cb[i], c1.cpu().numpy()), i
            finally:
                P.p3mz_destroy(h)
            off += s.n
    finally:
        P.p3mz_batch_destroy(b)


def test_batch_replica_against_oracle(torch):
    """Mixed-mode batch: the smallest replicas against the FP64 oracle (force
    bar 1e-5, equal V-cycle counts) over a short trajectory."""
    from paper_2606_31379_amd import p3maze as P
    reps, systems = build(torch, 1)
    reps, systems = reps[:3], systems[:3]
    dev = torch.device("cuda")
    n = [s.n for s in systems]
    b = P.p3mz_batch_create([sys_params(P, r, 1) for r in reps], n, packed([s.charges for s in systems]))
    oracles = [O.Oracle(O.make_params(r.box, 0.30, 9.0, r.mesh, 4, tol=1e-8, coulomb_k=K_E), s.charges)
               for r, s in zip(reps, systems)]
    stream = torch.cuda.current_stream().cuda_stream
    try:
        pos = torch.zeros((sum(n), 3), dtype=torch.float64, device=dev)
        frc = torch.zeros_like(pos)
        for step in range(3):
            xs = [s.pos + step * 0.5 * s.vel for s in systems]
            pos.copy_(torch.from_numpy(packed(xs)))
            P.p3mz_batch_compute(b, pos.data_ptr(), frc.data_ptr(), None, stream)
            torch.cuda.synchronize()
            fb = frc.cpu().numpy()
            off = 0
            for i, o in enumerate(oracles):
                fo, _, _ = o.compute(xs[i])
                assert rel_rms(fb[off:off + n[i]], fo) <= 1e-5, (step, i)
                assert P.p3mz_batch_get_stats(b, i).cycles == o.stats().cycles, (step, i)
                off += n[i]
    finally:
        P.p3mz_batch_destroy(b)


def test_batch_errors(torch):
    from paper_2606_31379_amd import p3maze as P
    reps, systems = build(torch, 1)
    q = packed([s.charges for s in systems[:2]])
    n = [s.n for s in systems[:2]]
    with pytest.raises(P.P3MZError):   # precisions differ
        P.p3mz_batch_create([sys_params(P, reps[0], 0), sys_params(P, reps[1], 1)], n, q)
    bad = q.copy()
    bad[0] += 1.0
    with pytest.raises(P.P3MZError):   # a non-neutral system
        P.p3mz_batch_create([sys_params(P, reps[0], 1), sys_params(P, reps[1], 1)], n, bad)
    b = P.p3mz_batch_create([sys_params(P, reps[0], 1)], n[:1], q[: n[0]])   # a batch of one
    P.p3mz_batch_destroy(b)


def test_full_64_replica_batch_against_oracle(torch):
    """The whole batched workload: 64 NaCl replicas of 512-32,768 ions on
    16^3-64^3 meshes (632,472 ions), mixed precision, captured graphs.  A
    cold solve and one warm step along the velocities; on every replica the
    V-cycle counts equal the FP64 oracle's, and the forces on 64 seeded ions
    per replica are within the mixed-mode bar."""
    from paper_2606_31379_amd import p3maze as P
    w = configs.nacl_batch_64()
    systems = w.systems()
    n = [s.n for s in systems]
    assert len(n) == 64 and sum(n) == 632472
    rng = np.random.Generator(np.random.PCG64(77))
    targets = [np.sort(rng.choice(s.n, size=64, replace=False)) for s in systems]
    trajs = [[s.pos, s.pos + w.dt_fs * s.vel] for s in systems]
    ref = []
    for r, s, tr, tg in zip(w.replicas, systems, trajs, targets):
        o = O.Oracle(O.make_params(r.box, w.alpha, w.r_cut, r.mesh, w.order, tol=w.tol, predictor=w.predictor,
                                   coulomb_k=K_E), s.charges)
        o.set_sr_targets(tg)
        rows = []
        for x in tr:
            f, _, _ = o.compute(x)
            rows.append((f[tg], o.stats().cycles))
        o.close()
        ref.append(rows)
    print(f"oracle done for {len(systems)} replicas", flush=True)
    dev = torch.device("cuda")
    b = P.p3mz_batch_create([sys_params(P, r, 1) for r in w.replicas], n, packed([s.charges for s in systems]))
    try:
        pos = torch.zeros((sum(n), 3), dtype=torch.float64, device=dev)
        frc = torch.zeros_like(pos)
        for k in range(2):
            pos.copy_(torch.from_numpy(packed([tr[k] for tr in trajs])))
            P.p3mz_batch_compute(b, pos.data_ptr(), frc.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            fg = frc.cpu().numpy()
            off, worst = 0, 0.0
            for i, s in enumerate(systems):
                fr, cyc = ref[i][k]
                st = P.p3mz_batch_get_stats(b, i)
                assert st.graphs == 1
                assert st.cycles == cyc, (k, i, st.cycles, cyc)
                err = rel_rms(fg[off:off + s.n][targets[i]], fr)
                worst = max(worst, err)
                assert err <= 1e-5, (k, i, err)
                off += s.n
            print(f"step {k}: worst replica rel-RMS force error {worst:.2e}", flush=True)
    finally:
        P.p3mz_batch_destroy(b)


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_halfsweeps_run_to_completion(torch, precision):
    """The persistent-kernel form of a batch's finest-level half-sweeps (one
    launch, per-system device barriers; a measurement prototype, not on the
    step path) finishes every task without a wait giving up, and the batch
    still steps to the oracle-checked result afterwards."""
    from paper_2606_31379_amd import p3maze as P
    reps, systems = build(torch, precision)
    n = [s.n for s in systems]
    q = packed([s.charges for s in systems])
    stream = torch.cuda.current_stream().cuda_stream
    b = P.p3mz_batch_create([sys_params(P, r, precision) for r in reps], n, q)
    try:
        dev = torch.device("cuda")
        pos = torch.from_numpy(packed([s.pos for s in systems])).to(dev)
        P.p3mz_batch_compute(b, pos.data_ptr(), None, None, stream)
        for k in (1, 8):
            ms, by = P.p3mz_batch_kernel_bench(b, P.PERSIST_HALFSWEEP, k, stream)
            assert np.isfinite(ms) and ms > 0 and by > 0
        ms1, _ = P.p3mz_batch_kernel_bench(b, P.KERNELS["halfsweep"], 8, stream)
        print(f"per half-sweep: persistent {ms * 1e3:.1f} us, batched launches {ms1 * 1e3:.1f} us", flush=True)
    finally:
        P.p3mz_batch_destroy(b)
