"""Thin ctypes binding of the C ABI in ``include/p3maze.h``.

Argument marshalling only: every computation runs in the HIP library
``libp3maze.so``.  Device buffers are passed as raw pointers (e.g.
``tensor.data_ptr()`` of torch CUDA tensors) and streams as raw
``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``).
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libp3maze.so")

P3MZ_OK = 0
P3MZ_WARN_NOT_CONVERGED = 1
P3MZ_ERR_INVALID_ARG = -1
P3MZ_ERR_NOT_NEUTRAL = -2
P3MZ_ERR_MESH_SHAPE = -3
P3MZ_ERR_OUT_OF_MEMORY = -4
P3MZ_ERR_HIP = -5
P3MZ_ERR_NAN = -6
P3MZ_ERR_STATE = -7
P3MZ_ERR_DENSITY = -8
P3MZ_PREC_FP64 = 0
P3MZ_PREC_MIXED = 1
P3MZ_PREC_MIXED32 = 2
MESH_Q, MESH_QS, MESH_SIGMA_P, MESH_Y, MESH_PHI, MESH_PHI_PREV = range(6)

# every symbol include/p3maze.h declares
EXPORTS = ["p3mz_create", "p3mz_compute", "p3mz_get_mesh", "p3mz_get_potential", "p3mz_vcycle",
           "p3mz_vcycle_noalloc", "p3mz_get_stats",
           "p3mz_reset_history", "p3mz_save_state", "p3mz_load_state", "p3mz_md_run",
           "p3mz_set_graphs", "p3mz_set_timing", "p3mz_set_kernel_timer", "p3mz_get_kernel_timer",
           "p3mz_get_kernel_launches",
           "p3mz_kernel_bench", "p3mz_set_schedule", "p3mz_set_fused_levels",
           "p3mz_set_neighbor_list", "p3mz_get_neighbor_stats", "p3mz_set_thermostat", "p3mz_autotune",
           "p3mz_destroy", "p3mz_batch_create", "p3mz_batch_compute", "p3mz_batch_md_run", "p3mz_batch_step",
           "p3mz_batch_get_stats", "p3mz_batch_set_timing", "p3mz_batch_get_timing", "p3mz_batch_set_graphs",
           "p3mz_batch_kernel_bench", "p3mz_batch_destroy", "p3mz_status_string", "p3mz_last_error", "p3mz_version"]
KERNELS = {"halfsweep": 0, "outer": 1, "smooth": 2, "restrict": 3, "prolong": 4, "sweep0": 5,
           "tail": 6, "spread": 7, "gather": 8, "sr": 9, "sigma": 10, "phi": 11, "fused_down": 12,
           "fused_up": 13}
PERSIST_HALFSWEEP = 14   # batches only: half-sweeps in one persistent launch


class p3mz_params(C.Structure):
    _fields_ = [("box", C.c_double), ("alpha", C.c_double), ("r_cut", C.c_double),
                ("mesh", C.c_int32), ("order", C.c_int32), ("tol", C.c_double),
                ("tol_mode", C.c_int32), ("max_cycles", C.c_int32), ("predictor", C.c_int32),
                ("precision", C.c_int32), ("coulomb_k", C.c_double), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("excl_group", C.c_int32), ("stencil", C.c_int32)]


class p3mz_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("cold", C.c_int32),
                ("m_eff", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("K", C.c_int32), ("levels", C.c_int32), ("nu_smooth", C.c_double),
                ("thresh", C.c_double), ("norm_qs", C.c_double), ("res_hist", C.c_double * 65),
                ("e_sr", C.c_double), ("e_lr", C.c_double), ("e_self", C.c_double),
                ("e_total", C.c_double), ("steps", C.c_int64), ("graphs", C.c_int32),
                ("ms_mesh", C.c_double), ("ms_short_range", C.c_double), ("ms_spread", C.c_double),
                ("ms_solve", C.c_double), ("ms_gather", C.c_double), ("net_force", C.c_double * 3)]


class p3mz_mdterms(C.Structure):
    _fields_ = [("model", C.c_int32), ("bm_a", C.c_double), ("bm_rho", C.c_double),
                ("lj_eps", C.c_double), ("lj_sigma", C.c_double), ("k_bond", C.c_double),
                ("r0", C.c_double), ("k_angle", C.c_double), ("theta0", C.c_double),
                ("force_to_acc", C.c_double), ("mv2_to_energy", C.c_double)]


class p3mz_tune_result(C.Structure):
    _fields_ = [("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("smooth_tile", C.c_int32),
                ("n_candidates", C.c_int32), ("ms_best", C.c_double), ("ms_default", C.c_double),
                ("ms_smooth", C.c_double), ("cand_nu_pre", C.c_int32 * 16), ("cand_nu_post", C.c_int32 * 16),
                ("cand_cycles", C.c_int32 * 16), ("cand_ms", C.c_double * 16),
                ("cand_ms_cycle", C.c_double * 16), ("cand_cycles_frac", C.c_double * 16),
                ("cand_expected_ms", C.c_double * 16)]


SMOOTH_TILES = 7


class P3MZError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_31379_amd.build`"
                          " (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    sig = {
        "p3mz_create": ([C.POINTER(p3mz_params), C.c_int64, dp, C.POINTER(vp)], C.c_int),
        "p3mz_compute": ([vp, vp, vp, vp, vp], C.c_int),
        "p3mz_get_mesh": ([vp, C.c_int32, vp, vp], C.c_int),
        "p3mz_get_potential": ([vp, vp, vp], C.c_int),
        "p3mz_vcycle": ([vp, vp, vp, vp], C.c_int),
        "p3mz_vcycle_noalloc": ([C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp], C.c_int),
        "p3mz_get_stats": ([vp, C.POINTER(p3mz_stats)], C.c_int),
        "p3mz_reset_history": ([vp], C.c_int),
        "p3mz_save_state": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
        "p3mz_load_state": ([vp, vp, C.c_size_t], C.c_int),
        "p3mz_md_run": ([vp, vp, vp, vp, C.POINTER(p3mz_mdterms), C.c_double, C.c_int32, vp, vp, vp],
                        C.c_int),
        "p3mz_set_graphs": ([vp, C.c_int32], C.c_int),
        "p3mz_set_timing": ([vp, C.c_int32], C.c_int),
        "p3mz_kernel_bench": ([vp, C.c_int32, C.c_int32, vp, dp, dp], C.c_int),
        "p3mz_set_kernel_timer": ([vp, C.c_int32], C.c_int),
        "p3mz_get_kernel_timer": ([vp, dp, C.POINTER(C.c_int64), dp], C.c_int),
        "p3mz_get_kernel_launches": ([vp, C.c_int32, C.POINTER(C.c_float), dp, ip], C.c_int),
        "p3mz_set_schedule": ([vp, C.c_int32, C.c_int32, C.c_int32], C.c_int),
        "p3mz_set_fused_levels": ([vp, C.c_int32], C.c_int),
        "p3mz_set_neighbor_list": ([vp, C.c_double, C.c_int32], C.c_int),
        "p3mz_set_thermostat": ([vp, C.c_double, C.c_double, C.c_uint64], C.c_int),
        "p3mz_get_neighbor_stats": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
        "p3mz_autotune": ([vp, vp, C.c_int32, vp, C.POINTER(p3mz_tune_result)], C.c_int),
        "p3mz_destroy": ([vp], None),
        "p3mz_batch_create": ([C.c_int32, C.POINTER(p3mz_params), C.POINTER(C.c_int64), dp, C.POINTER(vp)], C.c_int),
        "p3mz_batch_compute": ([vp, vp, vp, vp, vp], C.c_int),
        "p3mz_batch_md_run": ([vp, vp, vp, vp, C.POINTER(p3mz_mdterms), C.c_double, C.c_int32, vp, vp, vp],
                              C.c_int),
        "p3mz_batch_step": ([vp, vp, vp, vp, C.POINTER(p3mz_mdterms), C.c_double, vp, vp, vp, vp], C.c_int),
        "p3mz_batch_get_stats": ([vp, C.c_int32, C.POINTER(p3mz_stats)], C.c_int),
        "p3mz_batch_set_timing": ([vp, C.c_int32], C.c_int),
        "p3mz_batch_get_timing": ([vp, dp, dp, C.POINTER(C.c_int32)], C.c_int),
        "p3mz_batch_set_graphs": ([vp, C.c_int32], C.c_int),
        "p3mz_batch_kernel_bench": ([vp, C.c_int32, C.c_int32, vp, dp, dp], C.c_int),
        "p3mz_batch_destroy": ([vp], None),
        "p3mz_status_string": ([C.c_int], C.c_char_p),
        "p3mz_last_error": ([], C.c_char_p),
        "p3mz_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _check(code: int, where: str) -> int:
    if code < 0:
        raise P3MZError(code, where, lib.p3mz_last_error().decode())
    return code


# --- same names as the C ABI ------------------------------------------------
def p3mz_create(params: p3mz_params, charges_host) -> int:
    """charges_host: contiguous float64 numpy array. Returns the context handle."""
    h = C.c_void_p()
    _check(lib.p3mz_create(C.byref(params), int(charges_host.size),
                           charges_host.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
           "p3mz_create")
    return h.value


def p3mz_compute(ctx: int, pos_dev: int, force_dev: int | None, energy_dev: int | None,
                 stream: int | None = None) -> int:
    return _check(lib.p3mz_compute(ctx, pos_dev, force_dev, energy_dev, stream), "p3mz_compute")


def p3mz_get_mesh(ctx: int, which: int, out_dev: int, stream: int | None = None) -> int:
    return _check(lib.p3mz_get_mesh(ctx, which, out_dev, stream), "p3mz_get_mesh")


def p3mz_get_potential(ctx: int, phi_dev: int, stream: int | None = None) -> int:
    return _check(lib.p3mz_get_potential(ctx, phi_dev, stream), "p3mz_get_potential")


def p3mz_vcycle(ctx: int, r_dev: int, e_dev: int, stream: int | None = None) -> int:
    return _check(lib.p3mz_vcycle(ctx, r_dev, e_dev, stream), "p3mz_vcycle")


def p3mz_vcycle_noalloc(mesh: int, precision: int, nu_pre: int, nu_post: int, r_dev: int, e_dev: int,
                        stream: int | None = None) -> int:
    return _check(lib.p3mz_vcycle_noalloc(mesh, precision, nu_pre, nu_post, r_dev, e_dev, stream),
                  "p3mz_vcycle_noalloc")


def p3mz_get_stats(ctx: int) -> p3mz_stats:
    st = p3mz_stats()
    _check(lib.p3mz_get_stats(ctx, C.byref(st)), "p3mz_get_stats")
    return st


def p3mz_reset_history(ctx: int) -> int:
    return _check(lib.p3mz_reset_history(ctx), "p3mz_reset_history")


def p3mz_save_state(ctx: int) -> bytes:
    n = C.c_size_t(0)
    _check(lib.p3mz_save_state(ctx, None, C.byref(n)), "p3mz_save_state")
    buf = C.create_string_buffer(n.value)
    _check(lib.p3mz_save_state(ctx, buf, C.byref(n)), "p3mz_save_state")
    return buf.raw


def p3mz_load_state(ctx: int, blob: bytes) -> int:
    return _check(lib.p3mz_load_state(ctx, blob, len(blob)), "p3mz_load_state")


def p3mz_md_run(ctx: int, pos_dev: int, vel_dev: int, mass_dev: int, terms: p3mz_mdterms,
                dt: float, n_steps: int, energy_log_dev: int | None, cycles_log_dev: int | None,
                stream: int | None = None) -> int:
    return _check(lib.p3mz_md_run(ctx, pos_dev, vel_dev, mass_dev, C.byref(terms), dt, n_steps,
                                  energy_log_dev, cycles_log_dev, stream), "p3mz_md_run")


def p3mz_set_graphs(ctx: int, on: bool) -> int:
    return _check(lib.p3mz_set_graphs(ctx, int(on)), "p3mz_set_graphs")


def p3mz_kernel_bench(ctx: int, kernel_id: int, reps: int, stream: int | None = None) -> tuple[float, float]:
    """(mean launch milliseconds, algorithmic bytes per launch)."""
    ms, b = C.c_double(), C.c_double()
    _check(lib.p3mz_kernel_bench(ctx, kernel_id, reps, stream, C.byref(ms), C.byref(b)), "p3mz_kernel_bench")
    return ms.value, b.value


def p3mz_set_timing(ctx: int, on: bool) -> int:
    return _check(lib.p3mz_set_timing(ctx, int(on)), "p3mz_set_timing")


def p3mz_set_kernel_timer(ctx: int, kernel_id: int) -> int:
    return _check(lib.p3mz_set_kernel_timer(ctx, kernel_id), "p3mz_set_kernel_timer")


def p3mz_get_kernel_timer(ctx: int) -> tuple[float, int, float]:
    """(total event milliseconds, timed launches, total algorithmic bytes)."""
    ms, n, b = C.c_double(), C.c_int64(), C.c_double()
    _check(lib.p3mz_get_kernel_timer(ctx, C.byref(ms), C.byref(n), C.byref(b)), "p3mz_get_kernel_timer")
    return ms.value, n.value, b.value


def p3mz_get_kernel_launches(ctx: int, max_launches: int = 65536) -> tuple[list[float], list[float]]:
    """Per-launch (event milliseconds, algorithmic bytes) of the timed family, in launch order."""
    ms = (C.c_float * max_launches)()
    by = (C.c_double * max_launches)()
    n = C.c_int32()
    _check(lib.p3mz_get_kernel_launches(ctx, max_launches, ms, by, C.byref(n)), "p3mz_get_kernel_launches")
    return list(ms[:n.value]), list(by[:n.value])


def p3mz_set_schedule(ctx: int, nu_pre: int, nu_post: int, smooth_tile: int = 0) -> int:
    return _check(lib.p3mz_set_schedule(ctx, nu_pre, nu_post, smooth_tile), "p3mz_set_schedule")


def p3mz_set_fused_levels(ctx: int, max_edge: int) -> int:
    return _check(lib.p3mz_set_fused_levels(ctx, max_edge), "p3mz_set_fused_levels")


def p3mz_set_neighbor_list(ctx: int, skin: float, capacity: int = 0) -> int:
    return _check(lib.p3mz_set_neighbor_list(ctx, skin, capacity), "p3mz_set_neighbor_list")


def p3mz_set_thermostat(ctx: int, gamma: float, kt: float, seed: int = 0) -> int:
    return _check(lib.p3mz_set_thermostat(ctx, gamma, kt, seed), "p3mz_set_thermostat")


def p3mz_get_neighbor_stats(ctx: int) -> tuple[int, int, int]:
    """(list builds so far, atoms over capacity summed over builds, capacity)."""
    b, o, c = C.c_int64(), C.c_int64(), C.c_int32()
    _check(lib.p3mz_get_neighbor_stats(ctx, C.byref(b), C.byref(o), C.byref(c)), "p3mz_get_neighbor_stats")
    return b.value, o.value, c.value


def p3mz_autotune(ctx: int, frames_dev: int, n_frames: int, stream: int | None = None) -> p3mz_tune_result:
    """frames_dev: device pointer to [n_frames][n_atoms][3] float64 positions."""
    out = p3mz_tune_result()
    _check(lib.p3mz_autotune(ctx, frames_dev, n_frames, stream, C.byref(out)), "p3mz_autotune")
    return out


def p3mz_destroy(ctx: int) -> None:
    lib.p3mz_destroy(ctx)


def p3mz_batch_create(per_sys, n_atoms, charges_packed_host) -> int:
    """per_sys: sequence of p3mz_params; n_atoms: sequence of ints; charges: packed float64 numpy array."""
    n = len(per_sys)
    arr = (p3mz_params * n)(*per_sys)
    na = (C.c_int64 * n)(*[int(x) for x in n_atoms])
    h = C.c_void_p()
    _check(lib.p3mz_batch_create(n, arr, na, charges_packed_host.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
           "p3mz_batch_create")
    return h.value


def p3mz_batch_compute(b: int, pos_dev: int, force_dev: int | None, energies_dev: int | None,
                       stream: int | None = None) -> int:
    return _check(lib.p3mz_batch_compute(b, pos_dev, force_dev, energies_dev, stream), "p3mz_batch_compute")


def p3mz_batch_md_run(b: int, pos_dev: int, vel_dev: int, mass_dev: int, terms: p3mz_mdterms, dt: float,
                      n_steps: int, energy_log_dev: int | None, cycles_log_dev: int | None,
                      stream: int | None = None) -> int:
    return _check(lib.p3mz_batch_md_run(b, pos_dev, vel_dev, mass_dev, C.byref(terms), dt, n_steps, energy_log_dev,
                                        cycles_log_dev, stream), "p3mz_batch_md_run")


def p3mz_batch_step(b: int, pos_dev: int, vel_dev: int, mass_dev: int, terms: p3mz_mdterms, dt: float,
                    force_dev: int | None, energies_dev: int | None, cycles_dev: int | None,
                    stream: int | None = None) -> int:
    return _check(lib.p3mz_batch_step(b, pos_dev, vel_dev, mass_dev, C.byref(terms), dt, force_dev, energies_dev,
                                      cycles_dev, stream), "p3mz_batch_step")


def p3mz_batch_get_stats(b: int, sys: int) -> p3mz_stats:
    st = p3mz_stats()
    _check(lib.p3mz_batch_get_stats(b, sys, C.byref(st)), "p3mz_batch_get_stats")
    return st


def p3mz_batch_set_timing(b: int, on: bool) -> int:
    return _check(lib.p3mz_batch_set_timing(b, int(on)), "p3mz_batch_set_timing")


def p3mz_batch_get_timing(b: int) -> tuple[float, float, int]:
    """(mesh ms, short-range ms, ran from graphs) of the last batched step."""
    a, c, g = C.c_double(), C.c_double(), C.c_int32()
    _check(lib.p3mz_batch_get_timing(b, C.byref(a), C.byref(c), C.byref(g)), "p3mz_batch_get_timing")
    return a.value, c.value, g.value


def p3mz_batch_set_graphs(b: int, on: bool) -> int:
    return _check(lib.p3mz_batch_set_graphs(b, int(on)), "p3mz_batch_set_graphs")


def p3mz_batch_kernel_bench(b: int, kernel_id: int, reps: int, stream: int | None = None) -> tuple[float, float]:
    """(mean batched launch milliseconds, algorithmic bytes per launch over all systems)."""
    ms, by = C.c_double(), C.c_double()
    _check(lib.p3mz_batch_kernel_bench(b, kernel_id, reps, stream, C.byref(ms), C.byref(by)),
           "p3mz_batch_kernel_bench")
    return ms.value, by.value


def p3mz_batch_destroy(b: int) -> None:
    lib.p3mz_batch_destroy(b)


def p3mz_status_string(code: int) -> str:
    return lib.p3mz_status_string(code).decode()


def p3mz_last_error() -> str:
    return lib.p3mz_last_error().decode()


def p3mz_version() -> str:
    return lib.p3mz_version().decode()


def make_params(box, alpha, r_cut, mesh, order, tol=1e-8, tol_mode=0, max_cycles=50, predictor=3,
                precision=P3MZ_PREC_FP64, coulomb_k=1.0, nu_pre=2, nu_post=2,
                excl_group=0, stencil=0) -> p3mz_params:
    return p3mz_params(box, alpha, r_cut, mesh, order, tol, tol_mode, max_cycles, predictor,
                       precision, coulomb_k, nu_pre, nu_post, excl_group, stencil)
