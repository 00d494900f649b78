"""pe_bd_step_noalloc (the allocation-free entry point) against pe_bd_step:
the same state after the step, bit for bit, on two calls in a row, the
second with fewer bodies, beads and ions."""
import ctypes

import numpy as np
import pytest

from paper_2401_04865_amd import inputs

pytestmark = pytest.mark.gpu


def _state(ctx):
    return {k: ctx.sys_dev[k].clone() for k in ("bead_pos", "body_center", "body_quat", "ion_pos")}


def _step(B, ctx, s, fn_name, st, step_no):
    """Fresh solve and forces on the original configuration, then one step
    with the named entry point on a copy of the state."""
    ctx.load(s)
    ctx.solve()
    ctx.forces()
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t.numel() else None
    fn = getattr(B.lib(), fn_name)
    rc = fn(ctx.h, 1e-4, 1.0, 1.0, 20240109, step_no, P(st["bead_pos"]), P(st["body_center"]),
            P(st["body_quat"]), P(st["ion_pos"]))
    assert rc == B.PE_OK, B.lib().pe_last_error(ctx.h)
    return {k: v.cpu().numpy() for k, v in st.items()}


def test_noalloc_step_equals_workspace_step(gpu_lib):
    B = gpu_lib
    big = inputs.small_random_system(61, n_body=4, level=1, n_ion=40, L=8.0, sigma=0.16, mesh=(32, 32, 32),
                                     charges=[0.3, -0.2, 0.1, 0.0])
    small = inputs.small_random_system(62, n_body=2, level=1, n_ion=10, L=8.0, sigma=0.16, mesh=(32, 32, 32),
                                       charges=[0.2, -0.1])
    assert small.n_body < big.n_body and small.n_bead < big.n_bead and small.n_ion < big.n_ion
    for k, s in enumerate((big, small)):
        p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, precision=B.PE_MIXED)
        ctx = B.Context(p).load(s)
        ref = _step(B, ctx, s, "pe_bd_step", _state(ctx), 7 + k)
        got = _step(B, ctx, s, "pe_bd_step_noalloc", _state(ctx), 7 + k)
        for name in ref:
            assert np.array_equal(ref[name], got[name]), name
        # the step moved something
        assert not np.array_equal(ref["bead_pos"], s.bead_pos)
        ctx.close()


def test_noalloc_rejects_more_bodies_than_its_array(gpu_lib):
    """Argument checks come before any launch: a null state with bodies
    present is refused, and so is a call before any force pass."""
    B = gpu_lib
    s = inputs.small_random_system(63, n_body=2, level=1, n_ion=4, L=8.0, mesh=(32, 32, 32))
    p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8)
    ctx = B.Context(p).load(s)
    z = ctypes.c_void_p(0)
    assert B.lib().pe_bd_step_noalloc(ctx.h, 1e-4, 1.0, 1.0, 1, 0, z, z, z, z) == B.PE_ERR_STATE
    ctx.solve()
    ctx.forces()
    assert B.lib().pe_bd_step_noalloc(ctx.h, 1e-4, 1.0, 1.0, 1, 0, z, z, z, z) == B.PE_ERR_ARG
    ctx.close()
