"""Seeded synthetic inputs for the P3MaZe mesh step.

This module only draws particle configurations: positions, charges, masses,
velocities and box sizes.  It holds none of the method's arithmetic, so both
the HIP path and the CPU oracle can be fed from it without sharing any code.

Recipes (the paper's own systems are replaced by these synthetic stand-ins;
no dataset is involved):

* ``nacl``  -- molten-salt-like rock-salt ions: the first half Na (+1 e,
  22.99 amu), the second half Cl (-1 e, 35.45 amu), placed uniformly at
  random with a hard-core rejection on the minimum-image pair distance.
* ``water`` -- point-charge water: O (-0.82 e, 15.999 amu) placed uniformly
  at random with an O-O hard core, two H (+0.41 e, 1.008 amu) at a fixed
  O-H length and H-O-H angle with a uniformly random orientation, redrawn
  while any intermolecular pair is closer than a second hard core.
  Atoms are stored molecule by molecule as O, H, H.

Velocities are Maxwell-Boltzmann at the requested temperature with the
centre-of-mass velocity removed.  Units: Angstrom, e, amu, fs, K.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

KB_EV = 8.617333262e-5            # Boltzmann constant [eV/K]
EV_PER_AMU_A2_FS2 = 103.6427      # 1 amu*A^2/fs^2 expressed in eV
AMU_G = 1.66053906660e-24         # 1 amu in grams

NA_Q, CL_Q = 1.0, -1.0
NA_M, CL_M = 22.99, 35.45
O_Q, H_Q = -0.82, 0.41
O_M, H_M = 15.999, 1.008


@dataclasses.dataclass
class System:
    """One periodic particle system (host numpy arrays, float64)."""
    pos: np.ndarray        # [n, 3] Angstrom, inside [0, box)
    charges: np.ndarray    # [n] e
    masses: np.ndarray     # [n] amu
    vel: np.ndarray        # [n, 3] Angstrom/fs
    box: float             # cubic edge [Angstrom]
    kind: str              # "nacl" | "water" | "lattice"

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def density_g_cm3(self) -> float:
        return float(self.masses.sum() * AMU_G / (self.box * 1e-8) ** 3)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def hard_core_points(rng: np.random.Generator, n: int, box: float, dmin: float,
                     max_rounds: int = 400, progress=None) -> np.ndarray:
    """Uniform random points in a periodic cube, no pair closer than ``dmin``.

    Batched random sequential addition: each round draws a batch of uniform
    candidates, drops those within ``dmin`` (minimum image) of a point
    accepted in an earlier round, and of every conflicting pair inside the
    batch keeps only the lower-indexed candidate.  Accepted points keep their
    draw order.  The first test queries a KD-tree over most accepted points
    (rebuilt now and then) and small trees over the latest rounds' points.
    """
    chunks: list[np.ndarray] = []
    big, big_n = None, 0      # tree over the first big_n accepted points
    recent: list[cKDTree] = []   # one small tree per later round
    recent_n = 0
    have = 0
    for _ in range(max_rounds):
        need = n - have
        if need <= 0:
            break
        m = int(need * 1.5) + 64
        cand = rng.uniform(0.0, box, size=(m, 3))
        cand = np.minimum(cand, np.nextafter(box, 0.0))
        ok = np.ones(m, dtype=bool)
        if big is not None:
            d, _ = big.query(cand, k=1, distance_upper_bound=dmin, workers=-1)
            ok[d < dmin] = False
        for tree in recent:
            idx = np.nonzero(ok)[0]
            if idx.size == 0:
                break
            d, _ = tree.query(cand[idx], k=1, distance_upper_bound=dmin)
            ok[idx[d < dmin]] = False
        idx = np.nonzero(ok)[0]
        if idx.size > 1:
            ct = cKDTree(cand[idx], boxsize=box)
            pairs = ct.query_pairs(dmin, output_type="ndarray")
            if pairs.size:
                drop = np.unique(np.maximum(pairs[:, 0], pairs[:, 1]))
                keep = np.ones(idx.size, dtype=bool)
                keep[drop] = False
                idx = idx[keep]
        new = cand[idx[:need]]
        if progress is not None and (len(chunks) % 20 == 0 or have + new.shape[0] == n):
            progress(f"placed {have + new.shape[0]} of {n} points")
        if new.shape[0]:
            chunks.append(new)
            have += new.shape[0]
            recent_n += new.shape[0]
            if big is None or recent_n > big_n // 4 or len(recent) >= 16:
                big, big_n = cKDTree(np.concatenate(chunks, axis=0), boxsize=box), have
                recent, recent_n = [], 0
            else:
                recent.append(cKDTree(new, boxsize=box))
    if have < n:
        raise RuntimeError(f"could not place {n} points with separation {dmin} in box {box}")
    return np.concatenate(chunks, axis=0)


def maxwell_boltzmann(rng: np.random.Generator, masses: np.ndarray, temp_k: float) -> np.ndarray:
    """Velocities [A/fs] at temperature ``temp_k`` with zero total momentum."""
    s = np.sqrt(KB_EV * temp_k / (masses * EV_PER_AMU_A2_FS2))
    v = rng.standard_normal((masses.size, 3)) * s[:, None]
    vcm = (masses[:, None] * v).sum(axis=0) / masses.sum()
    return v - vcm


def nacl(n_ions: int, box: float, temp_k: float, seed: int, dmin: float = 2.0) -> System:
    """Molten-salt-like ions: indices [0, n/2) Na+, [n/2, n) Cl-."""
    if n_ions % 2:
        raise ValueError("n_ions must be even for a neutral salt")
    rng = _rng(seed)
    pos = hard_core_points(rng, n_ions, box, dmin)
    half = n_ions // 2
    q = np.concatenate([np.full(half, NA_Q), np.full(half, CL_Q)])
    m = np.concatenate([np.full(half, NA_M), np.full(half, CL_M)])
    vel = maxwell_boltzmann(rng, m, temp_k)
    return System(pos, q, m, vel, float(box), "nacl")


def _random_rotations(rng: np.random.Generator, k: int) -> np.ndarray:
    """Uniform random rotation matrices from normalised Gaussian quaternions."""
    qv = rng.standard_normal((k, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)


def water(n_mol: int, box: float, temp_k: float, seed: int, r_oh: float = 1.0,
          angle_deg: float = 109.47, d_oo: float = 2.4, d_inter: float = 1.2,
          max_rounds: int = 200, progress=None) -> System:
    """Point-charge water; atoms ordered O, H, H per molecule.  `progress`
    (optional) receives a short text now and then."""
    rng = _rng(seed)
    opos = hard_core_points(rng, n_mol, box, d_oo, progress=progress)
    half = math.radians(angle_deg) / 2.0
    tmpl = np.array([[0.0, 0.0, 0.0],
                     [r_oh * math.sin(half), 0.0, r_oh * math.cos(half)],
                     [-r_oh * math.sin(half), 0.0, r_oh * math.cos(half)]])
    rot = _random_rotations(rng, n_mol)
    mol_id = np.repeat(np.arange(n_mol), 3)

    def build(rmats):
        return opos[:, None, :] + np.einsum("mij,aj->mai", rmats, tmpl)

    pos = build(rot)

    def wrapped(p):
        f = np.mod(p.reshape(-1, 3), box)
        return np.minimum(f, np.nextafter(box, 0.0))

    def foreign_contacts(tree, tree_atoms, stale, atoms, pts):
        """(molecule, molecule) pairs of every intermolecular contact closer
        than d_inter between query atoms and the tree's atoms whose molecule
        is not stale.  Exact: an atom whose 8 nearest tree atoms all lie
        within d_inter is queried again by radius."""
        d, nb = tree.query(pts, k=8, distance_upper_bound=d_inter, workers=-1)
        hit = d < d_inter
        ja = tree_atoms[np.where(hit, nb, 0)]
        keep = hit & ~stale[mol_id[ja]] & (mol_id[ja] != mol_id[atoms][:, None])
        rows, cols = np.nonzero(keep)
        pa, pb = [mol_id[atoms[rows]]], [mol_id[ja[rows, cols]]]
        for i in np.nonzero(d[:, -1] < d_inter)[0]:
            js = tree_atoms[np.asarray(tree.query_ball_point(pts[i], d_inter), dtype=int)]
            js = js[~stale[mol_id[js]] & (mol_id[js] != mol_id[atoms[i]])]
            pa.append(np.full(js.size, mol_id[atoms[i]]))
            pb.append(mol_id[js])
        return np.concatenate(pa), np.concatenate(pb)

    # Contacts are found with a tree over the wrapped atoms as they were at
    # its build plus a small tree over the molecules re-drawn since then; the
    # big tree's entries of re-drawn molecules are stale and skipped.  Only
    # the molecules re-drawn in the last pass can have new contacts.
    flat = wrapped(pos)
    all_atoms = np.arange(3 * n_mol)
    static = cKDTree(flat, boxsize=box)
    moved = np.zeros(n_mol, dtype=bool)
    check = np.arange(n_mol)
    for _ in range(max_rounds):
        atoms = (3 * check[:, None] + np.arange(3)[None, :]).ravel()
        pa, pb = foreign_contacts(static, all_atoms, moved, atoms, flat[atoms])
        if moved.any():
            mv_atoms = np.nonzero(np.repeat(moved, 3))[0]
            qa, qb = foreign_contacts(cKDTree(flat[mv_atoms], boxsize=box), mv_atoms,
                                      np.zeros(n_mol, dtype=bool), atoms, flat[atoms])
            pa, pb = np.concatenate([pa, qa]), np.concatenate([pb, qb])
        bad = np.unique(np.concatenate([pa, pb]))
        if progress is not None:
            progress(f"orientation pass: {bad.size} molecules with contacts")
        if bad.size == 0:
            break
        rot[bad] = _random_rotations(rng, bad.size)
        pos[bad] = opos[bad, None, :] + np.einsum("mij,aj->mai", rot[bad], tmpl)
        flat.reshape(n_mol, 3, 3)[bad] = wrapped(pos[bad]).reshape(-1, 3, 3)
        moved[bad] = True
        check = bad
        if moved.sum() > n_mol // 4:
            static = cKDTree(flat, boxsize=box)
            moved[:] = False
    else:
        raise RuntimeError("could not orient water molecules without overlaps")
    pos = pos.reshape(-1, 3)
    q = np.tile([O_Q, H_Q, H_Q], n_mol)
    m = np.tile([O_M, H_M, H_M], n_mol)
    vel = maxwell_boltzmann(rng, m, temp_k)
    # positions stay unwrapped so molecules are whole; the mesh step wraps.
    return System(pos, q, m, vel, float(box), "water")


def rock_salt(n_cells: int, a: float, shift: float = 0.0) -> System:
    """Perfect rock-salt crystal of ``n_cells``^3 conventional cells (8 ions each).

    ``a`` is the conventional lattice constant (nearest-neighbour distance a/2);
    ``shift`` translates the whole crystal along (1,1,1).
    """
    base = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    cells = np.array([[i, j, k] for k in range(n_cells) for j in range(n_cells)
                      for i in range(n_cells)], dtype=float)
    na = (cells[:, None, :] + base[None]).reshape(-1, 3)
    cl = (cells[:, None, :] + base[None] + np.array([.5, 0, 0])).reshape(-1, 3)
    pos = np.concatenate([na, cl]) * a + shift
    box = n_cells * a
    pos = np.mod(pos, box)
    n = pos.shape[0]
    q = np.concatenate([np.full(n // 2, NA_Q), np.full(n // 2, CL_Q)])
    m = np.concatenate([np.full(n // 2, NA_M), np.full(n // 2, CL_M)])
    return System(pos, q, m, np.zeros_like(pos), float(box), "lattice")


def random_neutral(n: int, box: float, seed: int, dmin: float = 0.0) -> System:
    """Small test systems: random positions, alternating +-1 charges."""
    rng = _rng(seed)
    if dmin > 0:
        pos = hard_core_points(rng, n, box, dmin)
    else:
        pos = rng.uniform(0.0, box, size=(n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    if n % 2:
        q[-1] = 0.0
    m = np.full(n, 20.0)
    return System(pos, q, m, np.zeros_like(pos), float(box), "random")
