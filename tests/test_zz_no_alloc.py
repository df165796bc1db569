"""bf_energy_noalloc against bf_energy through the C-ABI: the same FP64 energy
(bitwise: the same kernels and partial counts, only the partials live in the
library's static scratch instead of a buffer of the problem), on two calls in
a row with the second on a smaller problem, and with the inversion flag set and
then cleared."""
import ctypes as C

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    from paper_2512_12151_amd import bfal
    return bfal


def energies(bf, pb):
    e, inv = C.c_double(), C.c_int32()
    st = bf.lib().bf_energy(pb.h, C.byref(e), C.byref(inv))
    assert st == bf.BF_OK
    e2, inv2 = C.c_double(), C.c_int32()
    st2 = bf.lib().bf_energy_noalloc(pb.h, C.byref(e2), C.byref(inv2))
    assert st2 == bf.BF_OK, bf.lib().bf_last_error(pb.ctx.h)
    return (e.value, inv.value), (e2.value, inv2.value)


def test_noalloc_energy_matches_bitwise(bf):
    ctx = bf.Context(0)
    big = bf.Problem.from_scene(ctx, scenes.medium())
    big.newton_step(tol=1e-3)
    small = bf.Problem.from_scene(ctx, scenes.tiny(lateral=(0.37, 0.21)))
    small.newton_step(tol=1e-3)
    for pb, name in ((big, "medium"), (small, "tiny")):   # larger first, then smaller
        (e, inv), (e2, inv2) = energies(bf, pb)
        print(f"{name}: bf_energy {e!r} inverted {inv}; noalloc {e2!r} inverted {inv2}", flush=True)
        assert inv == inv2 == 0
        assert np.isfinite(e) and e == e2
    # an inverted tet in x_hat: both report it; the next call on a valid state clears it
    sc = scenes.tiny()
    xh = sc["x_hat"].copy()
    t0 = sc["tets"][100]
    xh[t0[0]] = xh[t0[1]] + 2.0 * (xh[t0[1]] - xh[t0[0]])
    inv_pb = bf.Problem.from_scene(ctx, sc)
    inv_pb.newton_step(tol=1e-3)
    inv_pb.set_state(sc["x"], xh, sc["x_tilde"], sc["dt"])
    (e, inv), (e2, inv2) = energies(bf, inv_pb)
    assert inv == inv2 == 1 and e == e2 == np.inf
    (e, inv), (e2, inv2) = energies(bf, small)
    assert inv == inv2 == 0 and e == e2
    for pb in (big, small, inv_pb):
        pb.close()
    ctx.close()


def test_noalloc_needs_a_step_first(bf):
    ctx = bf.Context(0)
    pb = bf.Problem.from_scene(ctx, scenes.tiny())
    e, inv = C.c_double(), C.c_int32()
    assert bf.lib().bf_energy_noalloc(pb.h, C.byref(e), C.byref(inv)) == -8   # BF_ERR_STATE
    assert bf.lib().bf_energy_noalloc(pb.h, None, C.byref(inv)) == -1
    pb.close()
    ctx.close()
