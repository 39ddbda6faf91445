"""Entry points of the C ABI on the GPU beyond the parity cases: 16-bit
distributions round-trip through init_fields / fields to their storage
rounding, a handle moved to another stream continues bit for bit, batches
reject bad handle lists, a non-finite state is reported on a check step,
and the force history reports rows it no longer holds."""
import sys

import numpy as np
import pytest

import workloads as WL
from tests.helpers import gpu_solver, plate

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _state(shape, seed):
    rng = np.random.default_rng(seed)
    return 1 + 0.01 * rng.standard_normal(shape), 0.03 * rng.standard_normal((3,) + shape)


@pytest.mark.parametrize("storage,rel", [("fp32", 0.0), ("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_fdist_round_trip(storage, rel):
    """f - w is what is stored: reading back what was written gives f to the
    rounding of the deviation (exactly for FP32)."""
    _say("fdist round trip", storage)
    from oracle import lattice as OL
    bx = WL.box(37, 12, 9, [WL.PERIODIC] * 6, 0.7)
    rho, u = _state((9, 12, 37), 2)
    f = OL.equilibrium(rho, u)
    s = gpu_solver(bx, [], None, u0=u, rho0=rho, storage=storage)
    s.init_fields(fdist=f)
    g = s.fields("fdist")
    s.close()
    dev = np.abs(f - OL.W[:, None, None, None])
    err = np.abs(g - f)
    # float32 rounding of the deviation, then the 16-bit rounding
    assert np.all(err <= dev * (rel + 2.0 ** -23) + 1e-30)


def test_set_stream_continues_bitwise():
    import torch

    _say("set_stream")
    bx, wg, ph, u0 = plate(seed=3, nz=8)
    a = gpu_solver(bx, wg, ph, u0=u0)
    b = gpu_solver(bx, wg, ph, u0=u0)
    a.step(40)
    b.step(15)
    side = torch.cuda.Stream()
    b.set_stream(side)
    b.step(25)
    side.synchronize()
    np.testing.assert_array_equal(a.fields("fdist"), b.fields("fdist"))
    np.testing.assert_array_equal(a.forces(0, 40), b.forces(0, 40))
    a.close()
    b.close()


def test_batch_rejects_mixed_streams():
    import torch

    from paper_2102_01305_amd import _lib as L
    from paper_2102_01305_amd.solver import step_batch

    _say("step_batch, mixed streams")
    bx, wg, ph, u0 = plate(seed=3, nz=8)
    a = gpu_solver(bx, wg, ph, u0=u0)
    b = gpu_solver(bx, wg, ph, u0=u0)
    b.set_stream(torch.cuda.Stream())
    with pytest.raises(L.IbmlbmError):
        step_batch([a, b], 1)
    a.close()
    b.close()


def test_non_finite_state_is_reported_on_a_check_step():
    from paper_2102_01305_amd import _lib as L

    _say("divergence flag")
    bx = WL.box(32, 16, 8, [WL.PERIODIC] * 6, 0.7)
    rho, u = _state((8, 16, 32), 4)
    rho[3, 5, 7] = np.nan
    s = gpu_solver(bx, [], None, u0=u, rho0=rho, check_interval=2)
    s.step(4)
    with pytest.raises(L.IbmlbmError) as e:
        s.mass()
    assert e.value.code == L.EDIVERGED
    s.close()


def test_force_history_range():
    from paper_2102_01305_amd import _lib as L

    _say("force history ring")
    bx, wg, ph, u0 = plate(seed=1, nz=8)
    s = gpu_solver(bx, wg, ph, u0=u0, history_steps=16)
    s.step(40)
    f = s.forces(24, 16)
    assert f.shape == (16, 1, 8) and np.all(np.isfinite(f))
    for first, count in ((23, 2), (30, 11)):
        with pytest.raises(L.IbmlbmError) as e:
            s.forces(first, count)
        assert e.value.code == L.ERANGE
    s.close()
