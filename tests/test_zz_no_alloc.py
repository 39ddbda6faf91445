"""The entry point that allocates nothing, ibmlbm_create_noalloc, against
ibmlbm_create on the same solves: the caller's buffer holds only the two
lattice states and every other region comes from the library's static
device scratch.  Two calls in a row, the second on a smaller solve (the
scratch keeps the first one's contents), must give the same force history
and fields as the workspace entry point, bit for bit (the same kernels on
the same arguments).  A solve whose regions exceed the scratch is refused
with ENOMEM and a message naming the limit."""
import sys

import numpy as np
import pytest

from tests.helpers import clap_fling, plate

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(bx, wg, ph, u0, steps, step0, noalloc):
    from paper_2102_01305_amd.solver import Solver, complete_case

    gb, gw = complete_case(bx, wg, ph)
    u = u0.copy()
    if ph["kind"] == "clap_fling":
        u[0] += gb["u_in"][0]
    s = Solver(gb, gw, history_steps=256, noalloc=noalloc)
    s.init_fields(u=u, step0=step0)
    s.step(steps)
    out = (s.forces(step0, steps), s.fields("u"), s.fields("fdist"), s.markers("duB"))
    s.close()
    return out


def test_noalloc_matches_workspace_entry_point():
    cases = [("clap & fling 64x48x16, c=8, 70 steps from 150", clap_fling(seed=6, nx=64, ny=48, nz=16, chord=8.0,
                                                                           re=100.0, j=0.5, f=0.25), 70, 150),
             ("plate 64x32x8, 30 steps (smaller)", plate(seed=2, nz=8), 30, 0)]
    for name, (bx, wg, ph, u0), steps, step0 in cases:
        _say("no-alloc vs workspace:", name)
        ref = _run(bx, wg, ph, u0, steps, step0, False)
        got = _run(bx, wg, ph, u0, steps, step0, True)
        for a, b, what in zip(got, ref, ("forces", "u", "fdist", "duB")):
            assert np.array_equal(a, b), what


def test_noalloc_refuses_beyond_the_scratch():
    from paper_2102_01305_amd import _lib as L
    from paper_2102_01305_amd.solver import Solver, complete_case

    _say("no-alloc: history ring beyond the static scratch")
    bx, wg, ph, u0 = plate(seed=0, nz=8)
    gb, gw = complete_case(bx, wg, ph)
    with pytest.raises(L.IbmlbmError) as ei:
        Solver(gb, gw, history_steps=2_000_000, noalloc=True)   # 128 MB of history
    assert ei.value.code == L.ENOMEM
    assert "static scratch" in str(ei.value)
