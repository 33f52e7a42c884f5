"""C ABI checks that need no GPU: the library loads, exports every function the
header declares, sizes workspaces, and rejects bad arguments before it makes
any HIP call."""
import ctypes
import math
import os
import re

import pytest

import paper_1502_06216_amd as jk
from paper_1502_06216_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jko.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(jko_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return jk.load()


def test_header_declares_the_four_calls():
    names = _declared_functions()
    for n in ("jko_gibbs_apply", "jko_step", "jko_flow", "jko_backward", "jko_workspace_bytes"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # sizes implied by include/jko.h on x86-64
    assert ctypes.sizeof(nat.Grid) == 16
    assert ctypes.sizeof(nat.EnergyC) == 72
    assert ctypes.sizeof(nat.Params) == 48
    assert ctypes.sizeof(nat.Stats) == 48


def test_version_and_status_strings(lib):
    assert lib.jko_version() == nat.ABI_VERSION == 2
    assert lib.jko_status_string(0) == b"ok"
    assert b"capacity" in lib.jko_status_string(-5)
    assert lib.jko_status_string(123) == b"unknown status"


def test_workspace_bytes(lib):
    p = nat.make_params(1e-3, 1e-3, 300)
    small = jk.workspace_bytes((32, 32), jk.OP_STEP, 0, p)
    big = jk.workspace_bytes((256, 256), jk.OP_STEP, 0, p)
    assert 0 < small < big
    assert big >= 6 * 256 * 256 * 4
    flow = jk.workspace_bytes((256, 256), jk.OP_FLOW, 20, p)
    assert flow > big
    bwd = jk.workspace_bytes((64, 64), jk.OP_BACKWARD, 300, p)
    assert bwd >= 2 * 300 * 64 * 64 * 4
    assert jk.workspace_bytes((2000,), jk.OP_STEP, 0, p) == 0       # n > 1024
    assert jk.workspace_bytes((4, 4, 4, 4)[:3], 7, 0, p) == 0       # bad op
    # attraction: the stacked pair of couplings needs twice the fields; 1D/2D only
    att = jk.workspace_bytes((64, 64), nat.OP_ATTRACTION_STEP, 0, p)
    assert att > jk.workspace_bytes((64, 64), jk.OP_STEP, 0, p)
    assert jk.workspace_bytes((64, 64), nat.OP_ATTRACTION_FLOW, 4, p) > att
    assert jk.workspace_bytes((8, 8, 8), nat.OP_ATTRACTION_STEP, 0, p) == 0


def _call_step(lib, grid, energy, params, p_in=1, p_out=2, ws=16, nbytes=1 << 30, stats_dev=None):
    return lib.jko_step(ctypes.byref(grid), ctypes.byref(energy) if energy else None,
                        ctypes.byref(params) if params else None, ctypes.c_void_p(p_in),
                        ctypes.c_void_p(p_out), None, None if stats_dev is None else ctypes.c_void_p(stats_dev),
                        ctypes.c_void_p(ws), nbytes, None)


def test_argument_errors_before_any_launch(lib):
    """Validation happens on the host before any HIP call, so these run without
    a GPU (the pointers are never dereferenced)."""
    en = jk.EnergySpec(kind="congestion", kappa_scalar=1.0).to_c((8, 8))
    prm = nat.make_params(1e-3, 1e-3, 10)
    g = nat.make_grid((8, 8))
    bad = nat.make_grid((8, 8))
    bad.ndim = 4
    assert _call_step(lib, bad, en, prm) == jk.JKO_ERR_INVALID
    assert b"ndim" in lib.jko_last_error()
    big = nat.make_grid((2048, 8))
    assert _call_step(lib, big, en, prm) == jk.JKO_ERR_INVALID
    empty = nat.make_grid((0, 8))   # an empty grid is refused, not silently skipped
    assert _call_step(lib, empty, en, prm) == jk.JKO_ERR_INVALID
    assert b"n[k]" in lib.jko_last_error()
    for field, val in (("gamma", 0.0), ("gamma", math.nan), ("tau", -1.0), ("max_iters", 0),
                       ("check_every", 0), ("precision", 7), ("flags", 8), ("flags", -1)):
        p2 = nat.make_params(1e-3, 1e-3, 10)
        setattr(p2, field, val)
        assert _call_step(lib, g, en, p2) == jk.JKO_ERR_INVALID, field
    assert _call_step(lib, g, None, prm) == jk.JKO_ERR_INVALID
    assert _call_step(lib, g, en, None) == jk.JKO_ERR_INVALID
    assert _call_step(lib, g, en, prm, p_in=0) == jk.JKO_ERR_INVALID
    assert _call_step(lib, g, en, prm, p_in=5, p_out=5) == jk.JKO_ERR_INVALID
    # the device statistics record: 8-byte aligned, aliasing neither density
    assert _call_step(lib, g, en, prm, stats_dev=2) == jk.JKO_ERR_INVALID
    assert b"stats_dev" in lib.jko_last_error()
    assert _call_step(lib, g, en, prm, stats_dev=4100) == jk.JKO_ERR_INVALID
    assert _call_step(lib, g, en, prm, stats_dev=4096, ws=0) == jk.JKO_ERR_WORKSPACE
    e2 = jk.EnergySpec(kind="porous", m=1.0).to_c((8, 8))
    assert _call_step(lib, g, e2, prm) == jk.JKO_ERR_INVALID
    e3 = jk.EnergySpec(kind="congestion", kappa_scalar=-1.0).to_c((8, 8))
    assert _call_step(lib, g, e3, prm) == jk.JKO_ERR_INVALID
    e4 = nat.EnergyC()
    e4.kind = 9
    assert _call_step(lib, g, e4, prm) == jk.JKO_ERR_INVALID
    # binary congestion needs a finite capacity
    e5 = jk.EnergySpec(kind="binary_congestion", kappa_scalar=math.inf).to_c((8, 8))
    assert _call_step(lib, g, e5, prm) == jk.JKO_ERR_INVALID
    assert b"finite" in lib.jko_last_error()
    # attraction: a target, 1D/2D grids of at least 3 cells per axis
    e7 = jk.EnergySpec(kind="attraction", kappa_scalar=1.0).to_c((8, 8))
    assert _call_step(lib, g, e7, prm) == jk.JKO_ERR_INVALID
    assert b"target" in lib.jko_last_error()
    e7.target = ctypes.c_void_p(8)
    for grid_shape in ((8, 8, 8), (2, 8)):
        assert _call_step(lib, nat.make_grid(grid_shape), e7, prm) == jk.JKO_ERR_INVALID, grid_shape
    # generalised entropy: exponent >= 1, positive density scale
    for kw in ({"m": 0.5}, {"m": math.nan}, {"m": 1.5, "density_scale": 0.0}, {"m": 1.5, "coef_scalar": -1.0}):
        e6 = jk.EnergySpec(kind="gen_entropy", **kw).to_c((8, 8))
        assert _call_step(lib, g, e6, prm) == jk.JKO_ERR_INVALID, kw
    # workspace too small / missing
    assert _call_step(lib, g, en, prm, ws=0) == jk.JKO_ERR_WORKSPACE
    assert _call_step(lib, g, en, prm, nbytes=100) == jk.JKO_ERR_WORKSPACE
    assert b"needed" in lib.jko_last_error()


def test_gibbs_and_flow_and_backward_argument_errors(lib):
    g = nat.make_grid((8, 8))
    assert lib.jko_gibbs_apply(ctypes.byref(g), -1.0, 0, ctypes.c_void_p(1), ctypes.c_void_p(2),
                               ctypes.c_void_p(16), 1 << 20, None) == jk.JKO_ERR_INVALID
    assert lib.jko_gibbs_apply(ctypes.byref(g), 1e-3, 0, ctypes.c_void_p(1), ctypes.c_void_p(1),
                               ctypes.c_void_p(16), 1 << 20, None) == jk.JKO_ERR_INVALID
    en = jk.EnergySpec(kind="congestion", kappa_scalar=1.0).to_c((8, 8))
    prm = nat.make_params(1e-3, 1e-3, 10)
    assert lib.jko_flow(ctypes.byref(g), ctypes.byref(en), ctypes.byref(prm), 0, ctypes.c_void_p(1),
                        ctypes.c_void_p(2), None, None, ctypes.c_void_p(16), 1 << 30, None) == jk.JKO_ERR_INVALID
    iters = (ctypes.c_int32 * 2)(10, 0)
    assert lib.jko_backward(ctypes.byref(g), ctypes.byref(en), ctypes.byref(prm), 2, iters, ctypes.c_void_p(1),
                            ctypes.c_void_p(2), None, ctypes.c_void_p(3), ctypes.c_void_p(16), 1 << 30,
                            None) == jk.JKO_ERR_INVALID
    # no gradient through the binary (piecewise constant) prox
    binc = jk.EnergySpec(kind="binary_congestion", kappa_scalar=1.0).to_c((8, 8))
    assert lib.jko_backward(ctypes.byref(g), ctypes.byref(binc), ctypes.byref(prm), 2, iters, ctypes.c_void_p(1),
                            ctypes.c_void_p(2), None, ctypes.c_void_p(3), ctypes.c_void_p(16), 1 << 30,
                            None) == jk.JKO_ERR_INVALID
    assert b"piecewise constant" in lib.jko_last_error()
    # dL/dcoef of the generalised entropies needs the weight field
    gen = jk.EnergySpec(kind="gen_entropy", m=1.5).to_c((8, 8))
    assert lib.jko_backward(ctypes.byref(g), ctypes.byref(gen), ctypes.byref(prm), 2, iters, ctypes.c_void_p(1),
                            ctypes.c_void_p(2), ctypes.c_void_p(4), None, ctypes.c_void_p(16), 1 << 30,
                            None) == jk.JKO_ERR_INVALID
    assert b"coef" in lib.jko_last_error()
    ent = jk.EnergySpec(kind="entropy").to_c((8, 8))
    iters = (ctypes.c_int32 * 1)(10)
    # dL/dw only for congestion
    assert lib.jko_backward(ctypes.byref(g), ctypes.byref(ent), ctypes.byref(prm), 1, iters, ctypes.c_void_p(1),
                            ctypes.c_void_p(2), ctypes.c_void_p(4), None, ctypes.c_void_p(16), 1 << 30,
                            None) == jk.JKO_ERR_INVALID


def test_flags_field_and_binding():
    """jko_params.flags: the resident path and the 3D plane pass are the
    defaults; JKO_FLAG_NO_RESIDENT keeps one launch per application and
    JKO_FLAG_AXIS_PASSES three axis passes (the header names the bits)."""
    assert nat.make_params(1e-3, 1e-3).flags == 0
    assert nat.make_params(1e-3, 1e-3, resident=False).flags == nat.FLAG_NO_RESIDENT == 1
    assert nat.make_params(1e-3, 1e-3, planes=False).flags == nat.FLAG_AXIS_PASSES == 2
    assert nat.make_params(1e-3, 1e-3, resident=False, planes=False).flags == 3
    hdr = open(os.path.join(ROOT, "include", "jko.h")).read()
    assert "JKO_FLAG_NO_RESIDENT = 1" in hdr and "JKO_FLAG_AXIS_PASSES = 2" in hdr


def test_binding_refuses_cpu_tensors():
    import torch
    x = torch.zeros(8, 8)
    with pytest.raises(TypeError):
        jk.gibbs_apply(x, 1e-3)


def test_heat_domain_layout_and_workspace(lib):
    """The heat-kernel entry points: struct layout, workspace sizing (at
    least the upper-triangular 128 x 128 tiles of the operator: 79 tiles a
    side at 100 x 100), and argument errors refused on the host before any
    HIP call."""
    assert ctypes.sizeof(nat.HeatDomain) == 24
    d = nat.HeatDomain(100, 100, None, 10)
    nb = lib.jko_heat_workspace_bytes(ctypes.byref(d))
    assert nb >= 79 * 80 // 2 * 128 * 128 * 4
    assert lib.jko_heat_workspace_bytes(ctypes.byref(nat.HeatDomain(1, 9, None, 10))) > 0
    for n0, n1 in ((0, 5), (5, 0), (1025, 1025)):
        assert lib.jko_heat_workspace_bytes(ctypes.byref(nat.HeatDomain(n0, n1, None, 10))) == 0
    # above 2^16 cells (or on request) the products are solves: no stored operator
    big = lib.jko_heat_workspace_bytes(ctypes.byref(nat.HeatDomain(300, 300, None, 10)))
    assert 0 < big < 300 * 300 * 100
    solve = lib.jko_heat_workspace_bytes(ctypes.byref(nat.HeatDomain(100, 100, None, 10, 1)))
    assert 0 < solve < 100 * 100 * 100 < nb
    assert lib.jko_heat_workspace_bytes(None) == 0
    stream = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    # build: domain, L, gamma, workspace
    assert lib.jko_heat_build(None, 1e-3, fake, nb, stream) == jk.JKO_ERR_INVALID
    for L in (0, 1001):
        assert lib.jko_heat_build(ctypes.byref(nat.HeatDomain(10, 10, None, L)), 1e-3, fake, nb,
                                  stream) == jk.JKO_ERR_INVALID
    for gamma in (0.0, -1.0, math.inf, math.nan):
        assert lib.jko_heat_build(ctypes.byref(d), gamma, fake, nb, stream) == jk.JKO_ERR_INVALID
    assert lib.jko_heat_build(ctypes.byref(d), 1e-3, None, nb, stream) == jk.JKO_ERR_WORKSPACE
    assert lib.jko_heat_build(ctypes.byref(d), 1e-3, fake, nb - 1, stream) == jk.JKO_ERR_WORKSPACE
    assert lib.jko_heat_apply(ctypes.byref(d), fake, fake, fake, nb, stream) == jk.JKO_ERR_INVALID
    assert b"alias" in lib.jko_last_error()
    # flow: energy, precision, log domain, steps, pointers
    en = jk.EnergySpec(kind="congestion", kappa_scalar=1.0).to_c((100, 100))
    p_in, p_out = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)

    def flow(prm, e=en, n=1, a=p_in, b=p_out):
        return lib.jko_heat_flow(ctypes.byref(d), ctypes.byref(e), ctypes.byref(prm), n, a, b, None, fake, nb,
                                 stream)
    prm = nat.make_params(1e-3, 1e-2, 10)
    att = jk.EnergySpec(kind="attraction", kappa_scalar=1.0).to_c((100, 100))
    att.target = fake
    assert flow(prm, e=att) == jk.JKO_ERR_INVALID and b"attraction" in lib.jko_last_error()
    assert flow(nat.make_params(1e-3, 1e-2, 10, precision="split_bf16")) == jk.JKO_ERR_INVALID
    for thr in (0.0, 30.0, -math.inf):
        assert flow(nat.make_params(1e-3, 1e-2, 10, absorb_threshold=thr)) == jk.JKO_ERR_INVALID
    assert flow(prm, n=0) == jk.JKO_ERR_INVALID
    assert flow(prm, a=p_in, b=p_in) == jk.JKO_ERR_INVALID
    assert flow(prm, a=None) == jk.JKO_ERR_INVALID
    bad = nat.make_params(1e-3, 1e-2, 10)
    bad.max_iters = 0
    assert flow(bad) == jk.JKO_ERR_INVALID
