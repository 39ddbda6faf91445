"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/ibmlbm.h declares, and its host-only entry points validate input.
No call here touches a GPU."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibmlbm.h")


def _lib():
    from paper_2102_01305_amd import _lib as L
    return L, L.load()


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"IBMLBM_API[^;(]*?\b(ibmlbm_\w+)\s*\(", text))
    assert len(declared) >= 17
    bound = {name for name, _, _ in L.SIGNATURES}
    assert declared == bound, declared ^ bound
    for name in declared:
        assert hasattr(lib, name)


def test_struct_sizes_match_header_layout():
    L, _ = _lib()
    # int32 x9 (36) + pad 4 + doubles: tau, u_in[3], rho_out, body_force[3] (64)
    # + int32 x2 (8) + doubles u_ref, area_ref (16) + int64 (8)
    assert C.sizeof(L.Config) == 136
    assert C.sizeof(L.Wing) == 120
    assert L.Config.tau.offset == 40
    assert L.Wing.alpha_shape.offset == 64


def _cfg(bx, **kw):
    from paper_2102_01305_amd.solver import make_config
    return make_config(bx, **kw)


def _plate():
    from paper_2102_01305_amd.solver import complete_case
    bx, wg, ph = WL.plate_case()
    return complete_case(bx, wg, ph)


def test_workspace_bytes_and_validation():
    L, lib = _lib()
    from paper_2102_01305_amd.solver import make_wings
    bx, wg = _plate()
    c = _cfg(bx)
    w = make_wings(wg)
    lat = lib.ibmlbm_workspace_bytes(C.byref(c), 0, None)
    full = lib.ibmlbm_workspace_bytes(C.byref(c), 1, w)
    assert 0 < lat < full
    # two FP32 lattices of padded rows dominate: >= 2 * 19 * 4 bytes per cell
    assert lat >= 2 * 19 * 4 * 64 * 32 * 32
    for key, val in (("tau", 0.5), ("nx", 3)):
        bad = dict(bx)
        bad[key] = val
        assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(bad)), 0, None) == 0
        assert lib.ibmlbm_last_error(None)
    bad = dict(bx)
    bad["bc"] = [WL.PERIODIC, WL.WALL, 1, 1, 0, 0]
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(bad)), 0, None) == 0
    bad["bc"] = [0, 0, WL.VELOCITY, 1, 0, 0]
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(bad)), 0, None) == 0
    # a plate whose support would cross the inlet
    far = make_wings([dict(wg[0], hinge=[4.0, 15.5])])
    assert lib.ibmlbm_workspace_bytes(C.byref(c), 1, far) == 0
    assert b"leave the box" in lib.ibmlbm_last_error(None)
    # non-periodic span is rejected for extruded foils
    bad = dict(bx)
    bad["bc"] = [2, 3, 1, 1, 1, 1]
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(bad)), 1, w) == 0


def test_index_ranges_of_the_kernels_are_enforced():
    """Lattice rows (y, z) are 32-bit indices in the kernels and a row's 19
    population rows are addressed with 32-bit byte offsets: boxes beyond
    those ranges are refused before anything is allocated."""
    L, lib = _lib()
    bx, _ = _plate()
    ok = dict(bx, nx=(1 << 24) - 1, ny=4, nz=4)
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(ok)), 0, None) > 0
    for dims, msg in (((1 << 24, 4, 4), b"nx must be"), ((4, 1 << 16, 1 << 15), b"ny * nz")):
        bad = dict(bx, nx=dims[0], ny=dims[1], nz=dims[2])
        assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(bad)), 0, None) == 0
        assert msg in lib.ibmlbm_last_error(None)


def test_fp16_workspace_is_half_the_lattice():
    L, lib = _lib()
    bx, wg = _plate()
    b32 = lib.ibmlbm_workspace_bytes(C.byref(_cfg(bx, storage="fp32")), 0, None)
    b16 = lib.ibmlbm_workspace_bytes(C.byref(_cfg(bx, storage="bf16")), 0, None)
    assert b16 < 0.75 * b32


def test_clap_fling_wings_accepted_and_overlap_rejected():
    L, lib = _lib()
    from paper_2102_01305_amd.solver import complete_case, make_wings
    bx, wg, ph = WL.clap_fling_case()
    bx, wg = complete_case(bx, wg, ph)
    c = _cfg(bx)
    assert lib.ibmlbm_workspace_bytes(C.byref(c), 2, make_wings(wg)) > 0
    close = [dict(wg[0]), dict(wg[1], hinge=[wg[1]["hinge"][0], wg[0]["hinge"][1] - 2.0])]
    assert lib.ibmlbm_workspace_bytes(C.byref(c), 2, make_wings(close)) == 0
    assert b"support" in lib.ibmlbm_last_error(None)


def test_lattice_params_agree_with_the_paper_mapping():
    from paper_2102_01305_amd.solver import lattice_params
    p = lattice_params(100.0, 0.01, 0.25, 20.0)
    assert abs(p["tau"] - 0.53) < 1e-14
    assert abs(p["u_inf"] - 5e-4) < 1e-16
    assert abs(p["u_tip"] - 0.05) < 1e-16
    assert abs(p["period_steps"] - 2 * (2 * math.pi / 3) * 20 / 0.05) < 1e-9
    L, lib = _lib()
    t = C.c_double()
    assert lib.ibmlbm_lattice_params(-1.0, 0.0, 0.25, 20.0, 0.2, C.byref(t), None, None, None) == L.EINVAL


def test_plate_and_figure_eight_params():
    """Eq. 3 with Re = U c / nu: the plate workload (Re 100, u 0.02, c 10)
    has nu = 0.002 and tau = 0.506; the figure-eight stroke (Eq. 22, Re 75,
    U_tip 0.05, c 15, A0 = 2.5 c) has nu = 0.01, tau = 0.53 and the period
    pi A0 / U_tip = 2356.19 steps."""
    from paper_2102_01305_amd.solver import figure_eight_params, plate_params
    assert abs(plate_params(100.0, 0.02, 10.0)["tau"] - 0.506) < 1e-15
    p = figure_eight_params(75.0, 0.05, 15.0, 37.5)
    assert abs(p["tau"] - 0.53) < 1e-15
    assert abs(p["period_steps"] - math.pi * 37.5 / 0.05) < 1e-9
    L, lib = _lib()
    t = C.c_double()
    assert lib.ibmlbm_plate_params(100.0, 0.0, 10.0, C.byref(t)) == L.EINVAL
    assert lib.ibmlbm_figure_eight_params(75.0, 0.05, 15.0, -1.0, C.byref(t), None) == L.EINVAL


@pytest.mark.parametrize("chord,accepted", [(50.0, True), (60.0, True), (62.0, False)])
def test_marker_local_memory_limit(chord, accepted):
    """The marker kernels keep the perimeter records, a pivot row and column
    and the spread images in local memory (the perimeter block itself in
    registers, its inverse in L2), so a foil of up to the 128 perimeter
    markers a foil may have fits the 160 KB of a workgroup: a clap & fling
    pair at aspect ratio 5 with chord 60 (126 markers) is accepted, chord 62
    (130 markers) is refused at configuration time, not at the first step."""
    L, lib = _lib()
    from paper_2102_01305_amd.solver import complete_case, make_wings
    bx, wg, ph = WL.clap_fling_case(nx=400, ny=320, nz=8, chord=chord, re=100.0, j=0.01, f=0.25)
    gb, gw = complete_case(bx, wg, ph)
    n = lib.ibmlbm_workspace_bytes(C.byref(_cfg(gb)), len(gw), make_wings(gw))
    if accepted:
        assert n > 0
    else:
        assert n == 0
        assert b"perimeter markers" in lib.ibmlbm_last_error(None)


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2102_01305_amd.solver import Solver
    bx, wg = _plate()
    with pytest.raises(RuntimeError):
        Solver(bx, wg)


def test_single_hip_runtime_after_load():
    L, lib = _lib()
    import torch  # noqa: F401
    rts = L._hip_runtimes()
    assert len(rts) <= 1, rts


def test_one_layer_span_is_accepted_only_periodic():
    """nz = 1 with a periodic span is the 2D (D2Q9) scheme; short spans with
    z walls are rejected."""
    L, lib = _lib()
    bx, wg = _plate()
    one = dict(bx, nz=1)
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(one)), 0, None) > 0
    from paper_2102_01305_amd.solver import make_wings
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(one)), 1, make_wings(wg)) > 0
    walls = dict(bx, nz=2, bc=[WL.VELOCITY, WL.PRESSURE, WL.WALL, WL.WALL, WL.WALL, WL.WALL])
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(walls)), 0, None) == 0
    assert b"periodic" in lib.ibmlbm_last_error(None)


def test_span_longer_than_the_marker_block_is_rejected():
    """One block holds every span layer of a marker (its layer sums, B, the
    partial sums of the span solve) in local memory, so spans have a limit;
    the lattice alone has none, and the limit is named in the error."""
    L, lib = _lib()
    bx, wg = _plate()
    from paper_2102_01305_amd.solver import make_wings
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(dict(bx, nz=1024))), 1, make_wings(wg)) > 0
    long_span = dict(bx, nz=4096)
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(long_span)), 0, None) > 0
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(long_span)), 1, make_wings(wg)) == 0
    msg = lib.ibmlbm_last_error(None).decode()
    assert "span of 4096 layers" in msg
    top = int(msg.rsplit("at most ", 1)[1].rstrip(")"))
    assert 1024 <= top < 4096
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(dict(bx, nz=top))), 1, make_wings(wg)) > 0
    assert lib.ibmlbm_workspace_bytes(C.byref(_cfg(dict(bx, nz=top + 1))), 1, make_wings(wg)) == 0


@pytest.mark.parametrize("ds,accepted", [(1.0, True), (0.5, True), (0.3, False)])
def test_crowded_perimeter_is_refused_as_singular(ds, accepted):
    """Markers much closer than the lattice spacing make the perimeter block
    of the no-slip matrix (Eq. 18) singular in floating point: the plate foil
    (chord 10, thickness 2) with marker spacing 1 or 0.5 is accepted, with
    0.3 it is refused at configuration time with the reason."""
    L, lib = _lib()
    from paper_2102_01305_amd.solver import make_wings
    bx, wg = _plate()
    w = [dict(wg[0], ds=ds)]
    n = lib.ibmlbm_workspace_bytes(C.byref(_cfg(bx)), 1, make_wings(w))
    if accepted:
        assert n > 0
    else:
        assert n == 0
        assert b"singular" in lib.ibmlbm_last_error(None)
