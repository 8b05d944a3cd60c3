"""Helpers shared by the GPU tests: run the HIP library through its C ABI and
the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

K_E = 14.3996454784


def rel_rms(f, ref):
    den = np.sqrt((ref ** 2).sum())
    return float(np.sqrt(((f - ref) ** 2).sum()) / den) if den > 0 else float(np.sqrt((f ** 2).sum()))


class GpuCtx:
    """One library context plus torch device buffers for a fixed atom count."""

    def __init__(self, params, charges, torch):
        from paper_2606_31379_amd import p3maze as P
        self.P = P
        self.torch = torch
        self.n = int(charges.size)
        self.mesh = params.mesh
        self.h = P.p3mz_create(params, np.ascontiguousarray(charges, dtype=np.float64))
        dev = torch.device("cuda")
        self.pos = torch.zeros((self.n, 3), dtype=torch.float64, device=dev)
        self.force = torch.zeros((self.n, 3), dtype=torch.float64, device=dev)
        self.energy = torch.zeros(4, dtype=torch.float64, device=dev)
        self.mesh_buf = torch.zeros((self.mesh,) * 3, dtype=torch.float64, device=dev)

    def stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def compute(self, pos_np):
        self.pos.copy_(self.torch.from_numpy(np.ascontiguousarray(pos_np)))
        rc = self.P.p3mz_compute(self.h, self.pos.data_ptr(), self.force.data_ptr(),
                                 self.energy.data_ptr(), self.stream())
        self.torch.cuda.synchronize()
        return self.force.cpu().numpy().copy(), self.energy.cpu().numpy().copy(), rc

    def get_mesh(self, which):
        self.P.p3mz_get_mesh(self.h, which, self.mesh_buf.data_ptr(), self.stream())
        self.torch.cuda.synchronize()
        return self.mesh_buf.cpu().numpy().copy()

    def stats(self):
        return self.P.p3mz_get_stats(self.h)

    def vcycle(self, r):
        t = self.torch
        rr = t.from_numpy(np.ascontiguousarray(r)).cuda()
        ee = t.zeros_like(rr)
        self.P.p3mz_vcycle(self.h, rr.data_ptr(), ee.data_ptr(), self.stream())
        t.cuda.synchronize()
        return ee.cpu().numpy()

    def close(self):
        if self.h:
            self.P.p3mz_destroy(self.h)
            self.h = None


def params_pair(box, alpha, r_cut, mesh, order, tol=1e-8, precision=0, predictor=3, max_cycles=50,
                k_e=1.0, nu_pre=2, nu_post=2, excl_group=0, tol_mode=0, stencil=0):
    """Matching parameter structs for the library and the oracle."""
    from paper_2606_31379_amd import p3maze as P
    g = P.make_params(box, alpha, r_cut, mesh, order, tol=tol, tol_mode=tol_mode, max_cycles=max_cycles,
                      predictor=predictor, precision=precision, coulomb_k=k_e, nu_pre=nu_pre,
                      nu_post=nu_post, excl_group=excl_group, stencil=stencil)
    o = O.make_params(box, alpha, r_cut, mesh, order, tol=tol, tol_mode=tol_mode, max_cycles=max_cycles,
                      predictor=predictor, coulomb_k=k_e, nu_pre=nu_pre, nu_post=nu_post,
                      excl_group=excl_group, stencil=stencil)
    return g, o


def trajectory(system, steps, dt=0.5, seed=0):
    """Positions along straight-line motion with the system's velocities (A/fs)."""
    v = system.vel
    if not np.any(v):
        rng = np.random.default_rng(seed)
        v = rng.normal(scale=0.01, size=system.pos.shape)
    return [system.pos + k * dt * v for k in range(steps)]
