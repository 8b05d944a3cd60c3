"""Named synthetic workloads for the mesh step (no method arithmetic here).

Each workload fixes the physical recipe (``inputs``) and the electrostatic
control parameters of the paper's problem statement: box, Ewald splitting,
real-space cutoff, mesh, assignment order and solver tolerance.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

from . import inputs

K_E_EV_A = 14.3996454784   # Coulomb constant in eV*A/e^2
INPUTS_VERSION = "v1"      # bump when a recipe changes (invalidates cached systems)


@dataclasses.dataclass
class Workload:
    name: str
    kind: str               # "nacl" | "water"
    n_atoms: int
    box: float
    alpha: float
    r_cut: float
    mesh: int
    order: int
    tol: float
    temp_k: float
    seed: int
    md_steps: int = 1
    dt_fs: float = 0.5
    predictor: int = 3
    excl_group: int = 0     # 3 for water: O,H,H of one molecule are excluded pairs

    def generate(self, progress=None) -> inputs.System:
        if self.kind == "nacl":
            return inputs.nacl(self.n_atoms, self.box, self.temp_k, self.seed)
        if self.kind == "water":
            return inputs.water(self.n_atoms // 3, self.box, self.temp_k, self.seed, progress=progress)
        raise ValueError(self.kind)

    def system(self, progress=None) -> inputs.System:
        """The seeded system; systems of a million atoms or more are kept in
        an on-disk cache (directory P3MZ_INPUT_CACHE, default
        ~/.cache/p3maze/inputs) so that several processes share one draw."""
        if self.n_atoms < 1_000_000:
            return self.generate()
        d = os.environ.get("P3MZ_INPUT_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "p3maze", "inputs")
        path = os.path.join(d, f"{self.name}-seed{self.seed}-{INPUTS_VERSION}.npz")
        if os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            return inputs.System(z["pos"], z["charges"], z["masses"], z["vel"], float(z["box"]), str(z["kind"]))
        s = self.generate(progress)
        os.makedirs(d, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, pos=s.pos, charges=s.charges, masses=s.masses, vel=s.vel, box=s.box, kind=s.kind)
        os.replace(tmp, path)
        return s


def nacl_512() -> Workload:
    """512 molten-NaCl-like ions, L = 25.2 A, 32^3 mesh, order 4, FP64, one MD step."""
    return Workload("nacl-512-L25.2-m32-p4", "nacl", 512, 25.2, 0.30, 9.0, 32, 4, 1e-8,
                    1200.0, seed=1000, md_steps=1)


def water_3000() -> Workload:
    """1,000 point-charge water molecules (3,000 atoms) at L = 31.0 A, 64^3 mesh, order 4.

    The stated 3,000 molecules cannot fit a 31.0 A box at liquid density; the
    molecule count follows the linear-scaling recipe (62 A <-> 24,000 atoms)
    scaled by 1/8, giving 1.00 g/cm^3.
    """
    return Workload("water-3000-L31-m64-p4", "water", 3000, 31.0, 0.32, 9.0, 64, 4, 1e-8,
                    300.0, seed=2000, md_steps=100, excl_group=3)


def water_sweep(i: int) -> Workload:
    """Linear-scaling sweep: 24,000 / 192,000 / 1,536,000 atoms, meshes 64^3 / 128^3 / 256^3."""
    n = [24000, 192000, 1536000][i]
    box = [62.0, 124.0, 248.0][i]
    mesh = [64, 128, 256][i]
    return Workload(f"water-{n}-L{box:g}-m{mesh}-p4", "water", n, box, 0.32, 9.0, mesh, 4,
                    1e-6, 300.0, seed=3000 + i, md_steps=60, excl_group=3)


def water_large() -> Workload:
    """7,999,998-atom point-charge water, L = 431 A, 512^3 mesh, order 5."""
    return Workload("water-7999998-L431-m512-p5", "water", 7999998, 431.0, 0.30, 10.0, 512, 5,
                    1e-6, 300.0, seed=5000, md_steps=20, excl_group=3)


@dataclasses.dataclass
class Replica:
    n_atoms: int
    box: float
    mesh: int
    temp_k: float
    seed: int


def nacl_batch(n_sys: int = 64, seed: int = 4000) -> list[Replica]:
    """Replica recipe: atom counts log-uniform in [512, 32768] (even), box at
    1.55 g/cm^3 (L = 25.2 A * (n/512)^(1/3)), mesh 2^floor(log2(L/0.8)),
    temperature uniform in [1100, 1400] K."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_sys):
        n = int(2 * round(math.exp(rng.uniform(math.log(512), math.log(32768))) / 2))
        box = 25.2 * (n / 512.0) ** (1.0 / 3.0)
        mesh = 2 ** int(math.floor(math.log2(box / 0.8)))
        t = float(rng.uniform(1100.0, 1400.0))
        out.append(Replica(n, box, mesh, t, seed + 1 + i))
    return out


@dataclasses.dataclass
class BatchWorkload:
    """Batched NaCl replicas sharing the electrostatic control parameters."""
    name: str
    replicas: list
    alpha: float = 0.30
    r_cut: float = 9.0
    order: int = 4
    tol: float = 1e-8
    dt_fs: float = 0.5
    md_steps: int = 100
    predictor: int = 3

    @property
    def n_atoms(self) -> int:
        return sum(r.n_atoms for r in self.replicas)

    def systems(self) -> list:
        return [inputs.nacl(r.n_atoms, r.box, r.temp_k, r.seed) for r in self.replicas]


def nacl_batch_64() -> BatchWorkload:
    """64 NaCl replicas, log-uniform sizes in [512, 32768], meshes 16^3-64^3, order 4, tol 1e-8."""
    reps = nacl_batch(64)
    return BatchWorkload(f"nacl-batch64-{sum(r.n_atoms for r in reps)}", reps)


WORKLOADS = {
    "nacl-512": nacl_512,
    "water-3000": water_3000,
    "water-24000": lambda: water_sweep(0),
    "water-192000": lambda: water_sweep(1),
    "water-1536000": lambda: water_sweep(2),
    "water-7999998": water_large,
}
