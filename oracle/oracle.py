"""ctypes wrapper of the CPU FP64 oracle (``p3mz_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "p3mz_oracle.c")
LIB = os.path.join(HERE, "liboracle_p3mz.so")

MAX_CYCLES = 64
MAX_LEVELS = 16

OK, WARN_NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_NOT_NEUTRAL, ERR_MESH_SHAPE, ERR_OUT_OF_MEMORY = -1, -2, -3, -4
MESH_Q, MESH_QS, MESH_SIGMA_P, MESH_Y, MESH_PHI, MESH_PHI_PREV, MESH_Y_START = range(7)

KCAL_MOL_EV = 0.0433641
EV_PER_AMU_A2_FS2 = 103.6427


class Params(C.Structure):
    _fields_ = [("box", C.c_double), ("alpha", C.c_double), ("r_cut", C.c_double),
                ("mesh", C.c_int32), ("order", C.c_int32), ("tol", C.c_double),
                ("tol_mode", C.c_int32), ("max_cycles", C.c_int32), ("predictor", C.c_int32),
                ("coulomb_k", C.c_double), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("excl_group", C.c_int32), ("stencil", C.c_int32)]


class Plan(C.Structure):
    _fields_ = [("h", C.c_double), ("sigma", C.c_double), ("sigma_s2", C.c_double),
                ("nu_smooth", C.c_double), ("K", C.c_int32), ("levels", C.c_int32),
                ("nl", C.c_int32 * MAX_LEVELS)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("cold", C.c_int32),
                ("m_eff", C.c_int32), ("thresh", C.c_double), ("norm_qs", C.c_double),
                ("res_hist", C.c_double * (MAX_CYCLES + 1)),
                ("e_sr", C.c_double), ("e_lr", C.c_double), ("e_self", C.c_double),
                ("e_total", C.c_double), ("t_spread", C.c_double), ("t_solve", C.c_double),
                ("t_gather", C.c_double), ("t_sr", C.c_double), ("steps", C.c_int64)]


class MdTerms(C.Structure):
    _fields_ = [("model", C.c_int32), ("bm_a", C.c_double), ("bm_rho", C.c_double),
                ("lj_eps", C.c_double), ("lj_sigma", C.c_double), ("k_bond", C.c_double),
                ("r0", C.c_double), ("k_angle", C.c_double), ("theta0", C.c_double),
                ("force_to_acc", C.c_double), ("mv2_to_energy", C.c_double)]


def md_terms(model: str) -> MdTerms:
    """Non-electrostatic terms in eV / Angstrom / amu / fs units.

    water: flexible point-charge water, parameters of the paper's SI table of
    force-field parameters (LJ epsilon 0.1554253 kcal/mol, sigma 3.165492 A,
    r0 1.012 A, theta0 113.24 deg, k_b 1059.162 kcal/mol/A^2, k_a 75.90
    kcal/mol/rad^2), with the 1/2 k x^2 convention of that table's source.
    nacl: a stated stand-in Born-Mayer repulsion 4000 eV * exp(-r / 0.317 A)
    between all ion pairs (the paper's salt parameters are not printed).
    """
    t = MdTerms()
    t.force_to_acc = 1.0 / EV_PER_AMU_A2_FS2
    t.mv2_to_energy = EV_PER_AMU_A2_FS2
    if model == "none":
        t.model = 0
    elif model == "nacl":
        t.model = 1
        t.bm_a, t.bm_rho = 4000.0, 0.317
    elif model == "water":
        t.model = 2
        t.lj_eps = 0.1554253 * KCAL_MOL_EV
        t.lj_sigma = 3.165492
        t.k_bond = 1059.162 * KCAL_MOL_EV
        t.r0 = 1.012
        t.k_angle = 75.90 * KCAL_MOL_EV
        t.theta0 = np.deg2rad(113.24)
    else:
        raise ValueError(model)
    return t


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC",
                               "-shared", "-fopenmp", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_plan_make.argtypes = [C.POINTER(Params), C.POINTER(Plan)]
        L.orc_bspline.argtypes = [C.c_int, C.c_double]
        L.orc_bspline.restype = C.c_double
        L.orc_stencil_1d.argtypes = [C.c_int, C.c_int, C.c_double, ip, dp]
        L.orc_assign.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int64, dp, dp, dp]
        L.orc_smooth.argtypes = [C.c_int, C.c_int, C.c_double, dp]
        L.orc_apply_m.argtypes = [C.c_int, dp, dp]
        L.orc_apply_a19.argtypes = [C.c_int, dp, dp]
        L.orc_apply_a19.restype = None
        L.orc_apply_b.argtypes = [C.c_int, dp, dp]
        L.orc_apply_b.restype = None
        L.orc_rbgs.argtypes = [C.c_int, dp, dp, C.c_int]
        L.orc_restrict.argtypes = [C.c_int, dp, dp]
        L.orc_prolong_add.argtypes = [C.c_int, dp, dp]
        L.orc_coarsest.argtypes = [dp, dp]
        L.orc_vcycle_apply.argtypes = [C.c_void_p, dp, dp]
        L.orc_sr.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                             C.c_int32, C.POINTER(C.c_int64), C.c_int64, dp, dp]
        L.orc_ewald.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double, C.c_double,
                                C.c_double, dp, dp]
        L.orc_create.argtypes = [C.POINTER(Params), C.c_int64, dp, C.POINTER(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_destroy.restype = None
        L.orc_compute.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_get_stats.argtypes = [C.c_void_p, C.POINTER(Stats)]
        L.orc_set_sr_targets.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int64]
        L.orc_get_plan.argtypes = [C.c_void_p, C.POINTER(Plan)]
        L.orc_get_mesh.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_reset_history.argtypes = [C.c_void_p]
        L.orc_save_state.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]
        L.orc_load_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_md_run.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(MdTerms), C.c_double,
                                 C.c_int32, dp, ip]
        L.orc_nonelectrostatic.argtypes = [C.POINTER(MdTerms), C.c_int64, dp, C.c_double,
                                           C.c_double, dp, dp]
        u32p = C.POINTER(C.c_uint32)
        L.orc_set_thermostat.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_uint64]
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_thermo_normals.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int, dp]
        L.orc_thermo_normals.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(box, alpha, r_cut, mesh, order, tol=1e-8, tol_mode=0, max_cycles=50,
                predictor=3, coulomb_k=1.0, nu_pre=2, nu_post=2, excl_group=0, stencil=0) -> Params:
    return Params(box, alpha, r_cut, mesh, order, tol, tol_mode, max_cycles, predictor,
                  coulomb_k, nu_pre, nu_post, excl_group, stencil)


def plan(p: Params) -> Plan:
    out = Plan()
    rc = lib().orc_plan_make(C.byref(p), C.byref(out))
    if rc:
        raise OracleError(rc)
    return out


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


# ---- building blocks -------------------------------------------------------
def bspline(p: int, x: float) -> float:
    return lib().orc_bspline(p, x)


def stencil_1d(p: int, n: int, u: float):
    idx = np.zeros(p, dtype=np.int32)
    w = np.zeros(p)
    lib().orc_stencil_1d(p, n, u, idx.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return idx, w


def assign(p, n, box, pos, q):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros((n, n, n))
    lib().orc_assign(p, n, box, pos.shape[0], _dp(pos), _dp(q), _dp(out))
    return out  # [z][y][x]


def smooth(v, k_steps, nu):
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    lib().orc_smooth(v.shape[0], k_steps, nu, _dp(v))
    return v


def apply_m(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    lib().orc_apply_m(v.shape[0], _dp(v), _dp(out))
    return out


def apply_a19(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    lib().orc_apply_a19(v.shape[0], _dp(v), _dp(out))
    return out


def apply_b(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    lib().orc_apply_b(v.shape[0], _dp(v), _dp(out))
    return out


def rbgs(e, r, colour):
    e = np.array(e, dtype=np.float64, order="C", copy=True)
    r = np.ascontiguousarray(r, dtype=np.float64)
    lib().orc_rbgs(e.shape[0], _dp(e), _dp(r), colour)
    return e


def restrict(rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n = rho.shape[0]
    out = np.empty((n // 2,) * 3)
    lib().orc_restrict(n, _dp(rho), _dp(out))
    return out


def prolong_add(ec, e):
    ec = np.ascontiguousarray(ec, dtype=np.float64)
    e = np.array(e, dtype=np.float64, order="C", copy=True)
    lib().orc_prolong_add(ec.shape[0], _dp(ec), _dp(e))
    return e


def coarsest(r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    e = np.empty_like(r)
    lib().orc_coarsest(_dp(r), _dp(e))
    return e


def sr(pos, q, box, alpha, r_cut, k_e=1.0, excl_group=0, targets=None):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    if targets is None:
        nt, tp = pos.shape[0], None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = targets.size, targets.ctypes.data_as(C.POINTER(C.c_int64))
    f = np.zeros((nt, 3))
    e = np.zeros(nt)
    lib().orc_sr(pos.shape[0], _dp(pos), _dp(q), box, alpha, r_cut, k_e, excl_group, tp,
                 nt, _dp(f), _dp(e))
    return f, e


def ewald(pos, q, box, alpha, k_e=1.0, eps=1e-16):
    """Brute-force Ewald: returns ([E_real, E_recip, E_self], forces)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    e3 = np.zeros(3)
    f = np.zeros_like(pos)
    rc = lib().orc_ewald(pos.shape[0], _dp(pos), _dp(q), box, alpha, k_e, eps, _dp(e3), _dp(f))
    if rc:
        raise OracleError(rc)
    return e3, f


def nonelectrostatic(terms: MdTerms, pos, box, r_cut):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    f = np.zeros_like(pos)
    e = C.c_double(0.0)
    rc = lib().orc_nonelectrostatic(C.byref(terms), pos.shape[0], _dp(pos), box, r_cut, _dp(f),
                                    C.byref(e))
    if rc:
        raise OracleError(rc)
    return f, e.value


# ---- the mesh step -----------------------------------------------------------
class Oracle:
    """One oracle context: a system's charges plus the mesh-potential history."""

    def __init__(self, params: Params, charges):
        self.params = params
        self.charges = np.ascontiguousarray(charges, dtype=np.float64)
        self.n = self.charges.size
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(params), self.n, _dp(self.charges), C.byref(h))
        if rc:
            raise OracleError(rc)
        self._h = h
        self.mesh = params.mesh

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compute(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        f = np.zeros((self.n, 3))
        e = np.zeros(4)
        rc = lib().orc_compute(self._h, _dp(pos), _dp(f), _dp(e))
        if rc < 0:
            raise OracleError(rc)
        return f, e, rc

    def set_sr_targets(self, targets):
        """Pair term only for these atom indices (None: all atoms; empty: none)."""
        if targets is None:
            rc = lib().orc_set_sr_targets(self._h, None, -1)
        else:
            self._targets = np.ascontiguousarray(targets, dtype=np.int64)
            rc = lib().orc_set_sr_targets(self._h, self._targets.ctypes.data_as(C.POINTER(C.c_int64)),
                                          self._targets.size)
        if rc:
            raise OracleError(rc)

    def stats(self) -> Stats:
        s = Stats()
        lib().orc_get_stats(self._h, C.byref(s))
        return s

    def plan(self) -> Plan:
        p = Plan()
        lib().orc_get_plan(self._h, C.byref(p))
        return p

    def get_mesh(self, which: int):
        n = self.mesh
        out = np.empty((n, n, n))
        rc = lib().orc_get_mesh(self._h, which, _dp(out))
        if rc:
            raise OracleError(rc)
        return out

    def vcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        e = np.empty_like(r)
        lib().orc_vcycle_apply(self._h, _dp(r), _dp(e))
        return e

    def reset_history(self):
        lib().orc_reset_history(self._h)

    def save_state(self) -> bytes:
        n = C.c_size_t(0)
        lib().orc_save_state(self._h, None, C.byref(n))
        buf = C.create_string_buffer(n.value)
        rc = lib().orc_save_state(self._h, buf, C.byref(n))
        if rc:
            raise OracleError(rc)
        return buf.raw

    def load_state(self, blob: bytes):
        rc = lib().orc_load_state(self._h, blob, len(blob))
        if rc:
            raise OracleError(rc)

    def set_thermostat(self, gamma: float, kt: float, seed: int = 0):
        """OVRVO Langevin thermostat for md_run (gamma 0: none); restarts its step counter."""
        rc = lib().orc_set_thermostat(self._h, gamma, kt, seed)
        if rc:
            raise OracleError(rc)

    def md_run(self, pos, vel, mass, terms: MdTerms, dt, n_steps):
        pos = np.array(pos, dtype=np.float64, order="C", copy=True)
        vel = np.array(vel, dtype=np.float64, order="C", copy=True)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        elog = np.zeros((n_steps, 6))
        clog = np.zeros(n_steps, dtype=np.int32)
        rc = lib().orc_md_run(self._h, _dp(pos), _dp(vel), _dp(mass), C.byref(terms), dt, n_steps,
                              _dp(elog), clog.ctypes.data_as(C.POINTER(C.c_int32)))
        if rc < 0:
            raise OracleError(rc)
        return pos, vel, elog, clog, rc


def philox4x32_10(counter, key):
    """The oracle's Philox4x32-10: four 32-bit counter words, two key words -> four words."""
    c = (C.c_uint32 * 4)(*counter)
    k = (C.c_uint32 * 2)(*key)
    out = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def thermo_normals(seed: int, atom: int, step: int, half: int) -> np.ndarray:
    """The thermostat's three standard normals for (atom, step, end of the step)."""
    z = np.zeros(3)
    lib().orc_thermo_normals(seed, atom, step, half, _dp(z))
    return z
