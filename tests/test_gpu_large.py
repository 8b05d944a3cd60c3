"""GPU parity at the full sizes of the linear-scaling water sweep (24,000 /
192,000 / 1,536,000 atoms on 64^3 / 128^3 / 256^3) and of the large water
system (7,999,998 atoms on 512^3, order 5), in the launch configuration the
benchmark times (captured graphs).

The oracle computes the whole mesh step (assignment, smoothing, the V-cycle
solve, gather) for every atom, but the all-pairs short-range sum only for a
seeded sample of atoms; forces are compared on that sample, V-cycle counts
and the long-range energy on the whole system.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_31379_amd import configs

from .gpu_util import K_E, GpuCtx, params_pair, rel_rms

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-10
MIXED_BAR = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no HIP device")
    return _t


def sampled_parity(torch, w, precisions, steps, sample=512, schedule=(2, 2)):
    """V-cycle counts must be equal in every precision; with the FP32 charge
    source (2) a count may differ only where the oracle's residual lies
    within 1e-4 (relative) of its threshold.  `schedule` is the (nu_pre,
    nu_post) both sides run."""
    s = w.system(progress=lambda msg: print(f"[inputs] {msg}", flush=True))
    rng = np.random.Generator(np.random.PCG64(w.seed + 17))
    targets = np.sort(rng.choice(s.n, size=sample, replace=False))
    traj = [s.pos + k * w.dt_fs * s.vel for k in range(steps)]
    _, op = params_pair(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, k_e=K_E, excl_group=w.excl_group,
                        nu_pre=schedule[0], nu_post=schedule[1])
    o = O.Oracle(op, s.charges)
    o.set_sr_targets(targets)
    ref, ores, othr = [], [], []
    for x in traj:
        f, e, _ = o.compute(x)
        st = o.stats()
        ref.append((f[targets], st.cycles, e[1]))
        ores.append(list(st.res_hist))
        othr.append(st.thresh)
        print(f"oracle {w.name}: cycles {st.cycles} solve {st.t_solve:.1f}s", flush=True)
    o.close()
    for precision in precisions:
        gp, _ = params_pair(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, precision=precision, k_e=K_E,
                            excl_group=w.excl_group, nu_pre=schedule[0], nu_post=schedule[1])
        g = GpuCtx(gp, s.charges, torch)
        bar = FP64_BAR if precision == 0 else MIXED_BAR
        try:
            for k, x in enumerate(traj):
                fg, eg, _ = g.compute(x)
                st = g.stats()
                assert st.graphs == 1
                fr, cyc, e_lr = ref[k]
                err = rel_rms(fg[targets], fr)
                print(f"gpu {w.name} precision {precision} step {k}: cycles {st.cycles} err {err:.2e}", flush=True)
                assert err <= bar, (k, err)
                if precision == 2 and st.cycles != cyc:
                    c = min(st.cycles, cyc)
                    margin = abs(ores[k][c] - othr[k]) / othr[k]
                    print(f"  count differs ({st.cycles} vs {cyc}), oracle margin {margin:.2e}", flush=True)
                    assert margin < 1e-4, (k, st.cycles, cyc, margin)
                else:
                    assert st.cycles == cyc, (k, st.cycles, cyc)
                assert abs(eg[1] - e_lr) <= bar * abs(e_lr), k
        finally:
            g.close()


@pytest.mark.parametrize("i", [0, 1, 2])
def test_water_sweep_full_size(torch, i):
    sampled_parity(torch, configs.water_sweep(i), [0, 1, 2] if i < 2 else [1, 2, 0], steps=3)


def test_large_water_512_full_size(torch):
    """The large water system (7,999,998 atoms, 512^3, order 5, tolerance
    1e-6): two mesh steps (cold solve, then a warm step) in every precision,
    forces on 1,000 seeded atoms, V-cycle counts and the long-range energy of
    the whole system."""
    sampled_parity(torch, configs.water_large(), [1, 2, 0], steps=2, sample=1000)


@pytest.mark.parametrize("i", [2])
def test_water_sweep_schedule_1_2(torch, i):
    """The (1, 2) schedule the autotuner picks from 64^3 up: on 256^3 the
    single pre-smoothing sweep and the red-only restriction run as one walk
    over the fine planes (FP32 modes)."""
    sampled_parity(torch, configs.water_sweep(i), [1, 2, 0], steps=3, schedule=(1, 2))


def test_large_water_512_schedule_1_2(torch):
    """The benchmark's configuration: 512^3 with the (1, 2) schedule, FP32
    charge source, two steps."""
    sampled_parity(torch, configs.water_large(), [2, 1], steps=2, sample=1000, schedule=(1, 2))
