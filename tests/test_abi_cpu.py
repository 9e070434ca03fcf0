"""C ABI checks that need no GPU: the library loads, exports every function
include/bdem.h declares, and its host-side validation rejects bad inputs
before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2308_10459_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bdem.h")
LIB = os.path.join(ROOT, "paper_2308_10459_amd", "libbdem.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(bdem_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def B():
    if not os.path.exists(LIB):
        pytest.skip("libbdem.so not built")
    from paper_2308_10459_amd import bdem
    return bdem


def test_library_exports_every_declared_symbol(B):
    lib = C.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), f"{name} declared in bdem.h but not exported"
    assert set(names) == set(B.EXPORTED)


def test_struct_sizes_match_header_layout(B):
    # doubles first then int32s, natural alignment: the ctypes mirror must not pad differently
    assert C.sizeof(B.bdem_options) == 8 * (3 + 3 + 1 + 1 + 2 + 2 + 4) + 4 * 12
    assert C.sizeof(B.bdem_material) == 8 * 9 + 4 * 2
    assert C.sizeof(B.bdem_step_stats) == 4 * 4 + 8 + 8 * 3 + 8 * 8
    assert C.sizeof(B.bdem_tuning) == 4 * 6 + 8 * 3


def test_default_options(B):
    o = B.bdem_default_options()
    assert list(o.gravity) == [0.0, 0.0, -9.81]
    assert o.newton_rtol == 1e-8 and o.cg_rtol_max == 0.5 and o.max_cg == 2000
    assert o.precision == B.BDEM_PREC_FP64 and o.break_each_step == 1
    assert o.solver == B.BDEM_SOLVER_NEWTON
    assert o.integrator == B.BDEM_INTEGRATOR_EULER
    assert o.preconditioner == B.BDEM_PRECOND_BLOCK_JACOBI
    assert o.hessian == B.BDEM_HESS_GAUSS_NEWTON
    assert o.amg_refresh == 1


def test_workspace_bytes_scales_with_problem(B):
    small = S.make_block(nx=3, ny=3, nz=3)
    big = S.make_block(nx=6, ny=6, nz=6)
    o = B.scene_options(small)
    a, b = B.bdem_workspace_bytes(small, o), B.bdem_workspace_bytes(big, o)
    assert 0 < a < b
    om = B.scene_options(big, precision=B.BDEM_PREC_MIXED)
    assert B.bdem_workspace_bytes(big, om) < b


def _create_error(B, scene, **opt):
    with pytest.raises(B.BdemError) as ei:
        B.bdem_create(scene, B.scene_options(scene, **opt))
    return ei.value.code


@pytest.mark.parametrize("mutate,code", [
    ("self_bond", -1), ("duplicate", -1), ("index", -1), ("nonunit", -1), ("radius", -1),
    ("material", -1), ("cross_scene", -1), ("nan_pos", -4), ("coincident", -1), ("flag", -1),
    ("scene_order", -1)])
def test_create_rejects_invalid_inputs(B, mutate, code):
    sc = S.make_chain(n=4)
    if mutate == "self_bond":
        sc.ij = np.array([[0, 1], [2, 2]], dtype=np.int32)
    elif mutate == "duplicate":
        sc.ij = np.array([[0, 1], [1, 0]], dtype=np.int32)
    elif mutate == "index":
        sc.ij = np.array([[0, 7]], dtype=np.int32)
    elif mutate == "nonunit":
        sc.quat[1] = [0, 0, 0, 1.1]
    elif mutate == "radius":
        sc.radius[2] = 0.0
    elif mutate == "material":
        sc.pmat[0] = 3
    elif mutate == "cross_scene":
        sc.scene_id = np.array([0, 0, 1, 1], dtype=np.int32)
    elif mutate == "nan_pos":
        sc.pos[0, 0] = np.nan
    elif mutate == "coincident":
        sc.pos[1] = sc.pos[0]
    elif mutate == "flag":
        sc.flags[0] = 7
    elif mutate == "scene_order":
        sc.scene_id = np.array([1, 1, 0, 0], dtype=np.int32)
        sc.ij = np.array([[0, 1], [2, 3]], dtype=np.int32)
    assert _create_error(B, sc) == code


def test_create_rejects_friction_and_bad_limits(B):
    sc = S.make_chain(n=3)
    assert _create_error(B, sc, mu_s=-0.1) == -1
    assert _create_error(B, sc, k_self=float("nan")) == -1
    assert _create_error(B, sc, max_cg=0) == -1
    assert _create_error(B, sc, precision=5) == -1
    assert _create_error(B, sc, solver=2) == -1
    assert _create_error(B, sc, integrator=2) == -1
    assert _create_error(B, sc, preconditioner=2) == -1


def test_empty_scene_is_rejected(B):
    """No particles: no workspace size and INVALID from create, never a launch."""
    sc = S.make_chain(n=2)
    for k in ("pos", "quat", "vel", "qvel", "radius", "flags", "pmat"):
        setattr(sc, k, getattr(sc, k)[:0])
    sc.ij = np.zeros((0, 2), dtype=np.int32)
    assert sc.n == 0 and sc.nb == 0
    assert B.bdem_workspace_bytes(sc, B.scene_options(sc)) == 0
    assert _create_error(B, sc) == -1
