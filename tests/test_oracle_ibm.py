"""Pins of the oracle's immersed-boundary part.

Checks against facts the paper and the mathematics fix: values and sums of
the cosine kernel (Eq. 14), separability and diagonal of A (Eq. 18), the
single-marker closed form, adjointness of interpolation (Eq. 17) and
spreading (Eq. 15), the no-slip condition after the solve (Eq. 19), the
ellipse perimeter (complete elliptic integral), kinematics derivatives
(Eq. 23 / Eq. 20-21) and mirror symmetry of the clap & fling pair.
"""
import math

import numpy as np
import pytest
from scipy.special import ellipe

import workloads as WL
from oracle import ibm, params
from oracle import lattice as L
from oracle.sim import Sim


def test_delta_kernel_values():
    np.testing.assert_allclose(ibm.delta([0.0, 1.0, -1.0, 2.0, -2.0, 2.5, 3.0]),
                               [0.5, 0.25, 0.25, 0.0, 0.0, 0.0, 0.0], atol=1e-16)
    np.testing.assert_allclose(ibm.delta(0.5), (1 + math.sqrt(0.5)) / 4, rtol=1e-15)


def test_delta_kernel_sums():
    X = np.random.default_rng(0).uniform(-40, 40, 20000)
    j = np.arange(-50, 51)
    r = j[None, :] - X[:, None]
    d = ibm.delta(r)
    t = X - np.floor(X)
    np.testing.assert_allclose(d.sum(1), 1.0, atol=2e-15)                 # partition of unity
    np.testing.assert_allclose((d * d).sum(1), 3.0 / 8.0, atol=2e-15)     # sum of squares
    np.testing.assert_allclose((d * (-1.0) ** (j % 2)).sum(1), 0.0, atol=2e-15)  # even/odd split
    first = 0.5 - t + (np.sin(np.pi * t / 2) - np.cos(np.pi * t / 2)) / 2
    np.testing.assert_allclose((r * d).sum(1), first, atol=2e-15)


def _random_markers(m, dims, rng, margin=3.0):
    return np.stack([rng.uniform(margin, dims[d] - margin, m) for d in range(3)], axis=1)


def test_stencil_partition_of_unity_and_range():
    rng = np.random.default_rng(1)
    dims = (12, 10, 8)
    X = _random_markers(40, dims, rng, margin=0.0)
    nodes, w = ibm.stencil(X, dims, (True, True, True))
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-15)
    assert nodes.min() >= 0 and nodes.max() < 12 * 10 * 8
    with pytest.raises(ValueError):
        ibm.stencil(np.array([[0.5, 5.0, 4.0]]), dims, (False, True, True))


def test_interpolation_spreading_adjoint_and_conservative():
    rng = np.random.default_rng(2)
    dims = (10, 9, 8)
    N = 10 * 9 * 8
    X = _random_markers(30, dims, rng)
    nodes, w = ibm.stencil(X, dims, (False, False, True))
    dA = rng.uniform(0.5, 1.5, 30)
    g = rng.standard_normal(N)
    v = rng.standard_normal(30)
    Ig = ibm.interpolate(g, nodes, w)
    Sv = ibm.spread(v, dA, nodes, w, N)[0]
    assert abs((dA * v * Ig).sum() - (g * Sv).sum()) < 1e-12
    assert abs(Sv.sum() - (v * dA).sum()) < 1e-12
    np.testing.assert_allclose(ibm.interpolate(np.full(N, 2.5), nodes, w), 2.5, rtol=1e-15)


def _a1d(p, q):
    j = np.arange(math.floor(min(p, q)) - 4, math.ceil(max(p, q)) + 5)
    return float((ibm.delta(j - p) * ibm.delta(j - q)).sum())


def test_system_matrix_separable_closed_form():
    rng = np.random.default_rng(3)
    dims = (14, 14, 14)
    N = 14 ** 3
    X = rng.uniform(5, 9, size=(25, 3))
    dA = rng.uniform(0.5, 1.5, 25)
    nodes, w = ibm.stencil(X, dims, (False, False, False))
    M, A = ibm.system_matrix(nodes, w, dA, N)
    A = A.toarray()
    ref = np.array([[dA[l] * _a1d(X[k, 0], X[l, 0]) * _a1d(X[k, 1], X[l, 1]) * _a1d(X[k, 2], X[l, 2])
                     for l in range(25)] for k in range(25)])
    np.testing.assert_allclose(A, ref, atol=1e-15)
    np.testing.assert_allclose(np.diag(A), (3.0 / 8.0) ** 3 * dA, rtol=1e-14)


def test_single_marker_closed_form():
    # one marker moving with U through fluid at rest (rho = 1): the solve gives
    # du_B = U / ((3/8)^3 dA) and the force on the body is -(1024/27) U
    X = np.array([[6.3, 5.7, 6.1]])
    U = np.array([[0.01, -0.02, 0.005]])
    dA = np.array([0.8])
    dims = (12, 12, 12)
    N = 12 ** 3
    nodes, w = ibm.stencil(X, dims, (False, False, False))
    M, _ = ibm.system_matrix(nodes, w, dA, N)
    B = U - 0.0
    y = ibm.solve_dense(M, B)
    duB = y / dA[:, None]
    np.testing.assert_allclose(duB, U / ((3.0 / 8.0) ** 3 * dA[0]), rtol=1e-13)
    du = ibm.spread(duB.T, dA, nodes, w, N)
    np.testing.assert_allclose(ibm.interpolate(du, nodes, w).T, U, rtol=1e-13)
    f = ibm.wing_forces(np.ones(1), duB.T, dA, X, np.zeros(2), dict(sense=-1.0, chord=1.0), 1.0, 2.0)
    np.testing.assert_allclose(f[:3], -(1024.0 / 27.0) * U[0], rtol=1e-13)


def test_ellipse_perimeter_and_equal_spacing():
    for chord, thick in ((10.0, 2.0), (20.0, 4.0), (7.5, 1.0)):
        a, b = chord / 2, thick / 2
        P = 4 * a * ellipe(1 - (b / a) ** 2)
        assert abs(ibm.ellipse_arclength(a, b, 2 * math.pi) - P) < 1e-10 * P
        wg = WL.wing(chord, thick, (0, 0), 0.5, 0.0, 1.0, WL.ALPHA_CONST)
        ref, ds = ibm.perimeter_markers(wg)
        n = ref.shape[0]
        assert n == round(P)
        assert abs(ds - P / n) < 1e-12
        # marker points lie on the ellipse centred at the pivot (pivot_frac 1/2)
        np.testing.assert_allclose((ref[:, 0] / a) ** 2 + (ref[:, 1] / b) ** 2, 1.0, atol=1e-13)
        # consecutive markers are separated by equal arc length
        ph = np.unwrap(np.arctan2(ref[:, 1] / b, ref[:, 0] / a))
        arcs = [ibm.ellipse_arclength(a, b, p) for p in ph]
        np.testing.assert_allclose(np.diff(arcs), ds, rtol=1e-9)
    assert [ibm.perimeter_markers(WL.wing(c, c / 5, (0, 0), 1, 0, 1, 0))[0].shape[0]
            for c in (10, 20, 40)] == [21, 42, 84]


def _cf_wings():
    bx, wg, ph = WL.clap_fling_case()
    return params.complete_case(bx, wg, ph)


def test_clap_fling_kinematics_positions():
    bx, wg = _cf_wings()
    T = wg[0]["period_steps"]
    assert abs(T - 2 * (2 * math.pi / 3) * 20 / 0.05) < 1e-9
    up = wg[0]
    ref, _ = ibm.perimeter_markers(up)
    le = int(np.argmin(ref[:, 0]))              # leading edge: most upstream marker at t=0
    for t, al in ((0.0, 0.0), (T / 4, math.pi / 3), (T / 2, 0.0), (3 * T / 4, math.pi / 3)):
        X, U, Xh = ibm.marker_state(up, ref, 4, t)
        # the upper foil turns with sense -1: its leading edge rises with alpha
        lex = X[le * 4, 0]
        ley = X[le * 4, 1]
        assert abs(lex - (96 - 20 * math.cos(al))) < 1e-9
        assert abs(ley - (100.5 + 20 * math.sin(al))) < 1e-9
    # trailing edge marker sits on the hinge at all times
    X, U, Xh = ibm.marker_state(up, ref, 4, 123.0)
    np.testing.assert_allclose(X[0, :2], up["hinge"], atol=1e-12)


@pytest.mark.parametrize("shape", [WL.ALPHA_SIN, WL.ALPHA_ABS_SIN])
def test_kinematics_velocity_is_time_derivative(shape):
    wg = WL.wing(12.0, 2.4, (30.0, 20.0), 0.3, 0.2, -1.0, shape, alpha_mean=0.1,
                 alpha_amp=0.9, period_steps=400.0, phase=0.3, trans_amp=5.0, trans_angle=1.0)
    ref, _ = ibm.perimeter_markers(wg)
    h = 1e-4
    for t in (3.7, 55.2, 141.0, 333.3):
        X, U, _ = ibm.marker_state(wg, ref, 2, t)
        Xp, _, _ = ibm.marker_state(wg, ref, 2, t + h)
        Xm, _, _ = ibm.marker_state(wg, ref, 2, t - h)
        np.testing.assert_allclose((Xp - Xm) / (2 * h), U, atol=1e-8)


def test_abs_sin_kink_takes_forward_derivative():
    wg = WL.wing(10.0, 2.0, (0.0, 0.0), 1.0, 0.0, 1.0, WL.ALPHA_ABS_SIN,
                 alpha_amp=math.pi / 3, period_steps=100.0)
    for t in (0.0, 50.0, 100.0):
        al, ald = ibm.alpha(wg, t)
        assert abs(al) < 1e-12
        assert abs(ald - (math.pi / 3) * 2 * math.pi / 100) < 1e-15


def test_kronecker_solve_matches_dense_minimum_norm():
    rng = np.random.default_rng(4)
    nz = 16
    dims = (40, 30, nz)
    for th in (0.0, 0.37, -0.52, 1.2):
        wg = WL.wing(10.0, 2.0, (20.3, 15.1), 0.5, th, 1.0, WL.ALPHA_CONST)
        ref, ds = ibm.perimeter_markers(wg)
        X, U, _ = ibm.marker_state(wg, ref, nz, 0.0)
        m = X.shape[0]
        dA = np.full(m, ds)
        nodes, w = ibm.stencil(X, dims, (False, False, True))
        M, A = ibm.system_matrix(nodes, w, dA, 40 * 30 * nz)
        B = rng.standard_normal((m, 3))
        B = M @ B            # a consistent right-hand side (in the range of M)
        yd = ibm.solve_dense(M, B)
        yk = ibm.solve_block(M, B, tensor_shape=(ref.shape[0], nz))
        np.testing.assert_allclose(yk, yd, atol=1e-9 * np.abs(yd).max())
        np.testing.assert_allclose(M @ yk, B, atol=1e-10 * np.abs(B).max())
        # minimum norm: no component along the alternating span pattern
        alt = (-1.0) ** np.arange(nz)
        for c in range(3):
            Y = yk[:, c].reshape(-1, nz)
            assert np.abs(Y @ alt).max() < 1e-9 * np.abs(Y).max()


def test_alternating_span_mode_is_null():
    # why the minimum-norm reading is needed: A is singular for unit span spacing
    nz = 12
    X = np.stack([np.full(nz, 5.3), np.full(nz, 6.1), np.arange(nz) + 0.5], axis=1)
    nodes, w = ibm.stencil(X, (12, 12, nz), (False, False, True))
    M, _ = ibm.system_matrix(nodes, w, np.ones(nz), 12 * 12 * nz)
    alt = (-1.0) ** np.arange(nz)
    assert np.abs(M @ alt).max() < 1e-15


def _plate_sim(seed=0, nz=8):
    bx, wg, ph = WL.plate_case(nz=nz)
    bx, wg = params.complete_case(bx, wg, ph)
    u0 = WL.velocity_noise((nz, bx["ny"], bx["nx"]), seed)
    u0[0] += bx["u_in"][0]
    return Sim(bx, wg, u0=u0)


def test_no_slip_after_solve_and_force_identity():
    s = _plate_sim()
    s.run(3)
    Lr = s.last
    ucorr = (Lr["ustar"] + Lr["du"]).reshape(3, -1)
    res = ibm.interpolate(ucorr, Lr["nodes"], Lr["wts"]).T - Lr["U"]
    assert np.abs(res).max() < 1e-13
    # Eulerian total force = Lagrangian total force (the same kernel spreads
    # du_B and interpolates rho_B)
    Feul = (2 * Lr["rho"][None] * Lr["du"]).reshape(3, -1).sum(1)
    Flag = (2 * Lr["rhoB"][None] * Lr["duB"] * Lr["dA"][None]).sum(1)
    np.testing.assert_allclose(Feul, Flag, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(s.forces()[-1][0][:3], -Flag, rtol=1e-12, atol=1e-15)


def test_mirror_symmetric_pair():
    nx, ny, nz, c = 64, 48, 4, 8.0
    bx, wg, ph = WL.clap_fling_case(nx=nx, ny=ny, nz=nz, chord=c, re=100.0, j=0.5, f=0.25)
    bx, wg = params.complete_case(bx, wg, ph)
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = bx["u_in"][0]
    s = Sim(bx, wg, u0=u0)
    # start mid-stroke so the foils move
    s.n = 37
    s.run(6)
    h = s.forces()
    np.testing.assert_allclose(h[:, 0, 0], h[:, 1, 0], rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(h[:, 0, 1], -h[:, 1, 1], rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(h[:, 0, 4], h[:, 1, 4], rtol=1e-9, atol=1e-12)
    rho, u = s.fields()
    np.testing.assert_allclose(u[0], u[0][:, ::-1, :], atol=1e-13)
    np.testing.assert_allclose(u[1], -u[1][:, ::-1, :], atol=1e-13)


def test_lattice_params_clap_fling():
    p = params.clap_fling(100.0, 0.01, 0.25, 20.0)
    assert abs(p["u_tip"] - 0.05) < 1e-15
    assert abs(p["tau"] - 0.53) < 1e-14
    assert abs(p["u_inf"] - 5e-4) < 1e-16
    assert abs(p["period_steps"] - 1675.516081914556) < 1e-9
    p = params.plate(100.0, 0.02, 10.0)
    assert abs(p["tau"] - 0.506) < 1e-14


def test_figure_eight_kinematics_closed_form():
    """Eq. 20-22 at t = 0 and T/4: the centre sits at +A0/2 along the stroke
    plane, then crosses the hinge at the maximum speed pi A0 / T, which is
    the tip speed that defines Re; alpha goes from pi/4 to 0."""
    from oracle import params
    from oracle.ibm import alpha, hinge_motion

    bx, wg, ph = WL.figure_eight_case()
    ob, ow = params.complete_case(bx, wg, ph)
    w = ow[0]
    T = w["period_steps"]
    a0 = ph["a0"]
    beta = w["trans_angle"]
    e = np.array([math.cos(beta), math.sin(beta)])
    h0 = np.array(w["hinge"])
    X, V = hinge_motion(w, 0.0)
    assert np.allclose(X, h0 + 0.5 * a0 * e, atol=1e-12)
    assert np.allclose(V, 0.0, atol=1e-15)
    X, V = hinge_motion(w, T / 4.0)
    assert np.allclose(X, h0, atol=1e-12)
    assert np.allclose(V, -ph["u_tip"] * e, rtol=1e-12, atol=1e-15)
    assert alpha(w, 0.0)[0] == pytest.approx(math.pi / 4.0, abs=1e-15)
    assert alpha(w, T / 4.0)[0] == pytest.approx(0.0, abs=1e-14)
    assert ob["tau"] == pytest.approx(3.0 * ph["u_tip"] * ph["chord"] / ph["re"] + 0.5, rel=1e-15)


def test_single_marker_moment_closed_form():
    """Moment about the pivot (Sec. 3.7) of one marker moving with U through
    fluid at rest: the body force is -(1024/27) U (single-marker solve), so
    about a pivot at X - r the moment is M_z = r_x F_y - r_y F_x =
    -(1024/27)(r_x U_y - r_y U_x), and C_M = M_z / (0.5 u_ref^2 S chord)."""
    X = np.array([[6.3, 5.7, 6.1]])
    U = np.array([[0.01, -0.02, 0.005]])
    r = np.array([2.25, -1.5])
    dA = np.array([0.8])
    N = 12 ** 3
    nodes, w = ibm.stencil(X, (12, 12, 12), (False, False, False))
    M, _ = ibm.system_matrix(nodes, w, dA, N)
    duB = ibm.solve_dense(M, U) / dA[:, None]
    u_ref, area, chord = 0.05, 3.0, 2.5
    f = ibm.wing_forces(np.ones(1), duB.T, dA, X, X[0, :2] - r, dict(sense=1.0, chord=chord), u_ref, area)
    k = 1024.0 / 27.0
    mz = -k * (r[0] * U[0, 1] - r[1] * U[0, 0])
    np.testing.assert_allclose(f[3], mz, rtol=1e-13)
    np.testing.assert_allclose(f[7], mz / (0.5 * u_ref ** 2 * area * chord), rtol=1e-13)


def _translating_foil(pivot_frac, centre):
    # a foil with an even number of perimeter markers (22), chord along x,
    # translating with a uniform velocity through fluid at rest (Eq. 20 at
    # t = 0 with phase -pi/2: the pivot moves at trans_amp * 2 pi / T along
    # trans_angle); fully periodic box
    a = 5.0
    hinge = (centre[0] + a * (2.0 * pivot_frac - 1.0), centre[1])
    wg = [WL.wing(2 * a, 2.0, hinge, pivot_frac, 0.0, 1.0, WL.ALPHA_CONST, period_steps=400.0,
                  phase=-math.pi / 2, trans_amp=2.0, trans_angle=0.7, ds=0.95)]
    bx = WL.box(32, 32, 4, [WL.PERIODIC] * 6, 0.8, u_ref=0.03, area_ref=2 * a * 4)
    s = Sim(bx, wg)
    assert s.refs[0].shape[0] == 22
    s.step()
    return s.forces()[0, 0], a


def test_moment_of_translating_foil_about_centre_and_trailing_edge():
    """A point-symmetric marker set (ellipse with an even number of markers,
    centre on a lattice node of a periodic box) translating uniformly from
    rest has point-symmetric marker forces, so its moment about the centre
    vanishes while the force does not; about the trailing edge, a = c/2
    further along the chord, the moment is then M_c - a F_y = -a F_y
    (moment transfer between two points)."""
    fc, a = _translating_foil(0.5, (16.0, 16.0))
    ft, _ = _translating_foil(1.0, (16.0, 16.0))
    F = np.hypot(fc[0], fc[1])
    assert F > 1e-3
    np.testing.assert_allclose(ft[:3], fc[:3], rtol=1e-13)
    assert abs(fc[3]) <= 1e-12 * a * F
    np.testing.assert_allclose(ft[3], -a * fc[1], rtol=1e-12)
    qs = 0.5 * 0.03 ** 2 * (10.0 * 4)
    np.testing.assert_allclose(ft[7], ft[3] / (qs * 10.0), rtol=1e-13)
