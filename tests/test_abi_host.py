"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and rejects bad problems before touching
the device."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "p3maze.h")).read()
    return sorted(set(re.findall(r"\b(p3mz_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2606_31379_amd import p3maze as P
    declared = header_functions()
    assert set(declared) == set(P.EXPORTS)
    for name in declared:
        assert hasattr(P.lib, name), name
    assert P.p3mz_version().startswith("p3maze-gfx950")


def test_status_strings():
    from paper_2606_31379_amd import p3maze as P
    for code in range(-8, 2):
        assert P.p3mz_status_string(code) != "unknown status"


@pytest.mark.parametrize("kw,code", [
    (dict(mesh=12), -3), (dict(mesh=4), -3), (dict(mesh=24), -3),
    (dict(order=8), -1), (dict(order=1), -1),
    (dict(r_cut=6.0), -1), (dict(tol=0.0), -1), (dict(max_cycles=65), -1),
    (dict(predictor=4), -1),
])
def test_invalid_parameters_rejected_before_allocation(kw, code):
    from paper_2606_31379_amd import p3maze as P
    args = dict(box=10.0, alpha=0.5, r_cut=4.0, mesh=16, order=4)
    args.update(kw)
    params = P.make_params(**args)
    q = np.array([1.0, -1.0])
    with pytest.raises(P.P3MZError) as ei:
        P.p3mz_create(params, q)
    assert ei.value.code == code


def test_non_neutral_rejected():
    from paper_2606_31379_amd import p3maze as P
    with pytest.raises(P.P3MZError) as ei:
        P.p3mz_create(P.make_params(10.0, 0.5, 4.0, 16, 4), np.array([1.0, 1.0, -1.5]))
    assert ei.value.code == P.P3MZ_ERR_NOT_NEUTRAL


def test_mesh_too_coarse_for_sigma():
    from paper_2606_31379_amd import p3maze as P
    # sigma = 1/(sqrt2 * 2) = 0.35 < h*sqrt(p/6) at h = 1.25
    with pytest.raises(P.P3MZError) as ei:
        P.p3mz_create(P.make_params(10.0, 2.0, 4.0, 8, 4), np.array([1.0, -1.0]))
    assert ei.value.code == P.P3MZ_ERR_MESH_SHAPE


def test_product_package_never_uses_the_oracle():
    pat = re.compile(r"(import\s+oracle|from\s+oracle|p3mz_oracle|liboracle|orc_[a-z_]+\()")
    pkg = os.path.join(ROOT, "paper_2606_31379_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not pat.search(txt), f


def test_null_context_rejected_by_the_md_and_pair_options():
    """The neighbour-list and thermostat entry points check their arguments
    before any device call (no GPU needed)."""
    import ctypes as C
    from paper_2606_31379_amd import p3maze as P
    L = P.lib
    assert L.p3mz_set_neighbor_list(None, 0.5, 0) == P.P3MZ_ERR_INVALID_ARG
    assert L.p3mz_set_thermostat(None, 0.1, 0.025, 1) == P.P3MZ_ERR_INVALID_ARG
    b, o, c = C.c_int64(), C.c_int64(), C.c_int32()
    assert L.p3mz_get_neighbor_stats(None, C.byref(b), C.byref(o), C.byref(c)) == P.P3MZ_ERR_INVALID_ARG


def test_stencil_validated_before_allocation():
    from paper_2606_31379_amd import p3maze as P
    q = np.array([1.0, -1.0])
    for kw in (dict(order=6, stencil=1), dict(order=4, stencil=2), dict(order=4, stencil=-1)):
        with pytest.raises(P.P3MZError) as ei:
            P.p3mz_create(P.make_params(10.0, 0.5, 4.0, 16, **kw), q)
        assert ei.value.code == P.P3MZ_ERR_INVALID_ARG
