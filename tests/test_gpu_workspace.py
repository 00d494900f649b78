"""The caller-owned device workspace: the library's only device memory is
a region the caller registers (here a torch tensor), sized by
pe_workspace_size, grown by moving the live buffers into a new region."""
import ctypes

import numpy as np
import pytest

from paper_2401_04865_amd import inputs

pytestmark = pytest.mark.gpu


def _system():
    return inputs.small_random_system(41, n_body=3, level=1, n_ion=30, L=7.0, sigma=0.16, mesh=(32, 32, 32),
                                      charges=[0.4, -0.1, 0.0])


def test_solve_in_a_torch_workspace(gpu_lib):
    """Through the C ABI: size the workspace, register a torch tensor, load,
    solve; the result equals that of a context whose binding manages the
    workspace itself, and a region too small is refused with PE_ERR_NOMEM
    (the size it needed is then reported)."""
    import torch
    B = gpu_lib
    lib = B.lib()
    s = _system()
    p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-12)
    ref = B.Context(p).load(s).solve()["q"].cpu().numpy()

    h = ctypes.c_void_p()
    assert lib.pe_create(ctypes.byref(p), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                         ctypes.byref(h)) == B.PE_OK
    nbytes = ctypes.c_size_t()
    assert lib.pe_workspace_size(h, s.n_bead, s.n_body, s.n_ion, ctypes.byref(nbytes)) == B.PE_OK
    assert nbytes.value > 0
    dev = {k: torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64), device="cuda")
           for k, v in dict(bp=s.bead_pos, bs=s.bead_sigma, bc=s.body_center, bq=s.body_quat, Q=s.body_charge,
                            ip=s.ion_pos, iq=s.ion_charge, isg=s.ion_sigma).items()}
    off = np.ascontiguousarray(s.body_offsets, dtype=np.int64)
    e0 = (ctypes.c_double * 3)(*s.E0)
    P = lambda t: ctypes.c_void_p(t.data_ptr())

    def load():
        return lib.pe_set_system(h, s.n_body, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), P(dev["bp"]),
                                 P(dev["bs"]), P(dev["bc"]), P(dev["bq"]), P(dev["Q"]), s.n_ion, P(dev["ip"]),
                                 P(dev["iq"]), P(dev["isg"]), e0)
    # no region yet, then a region far too small: refused, and the need reported
    assert load() == B.PE_ERR_NOMEM
    tiny = torch.empty(4096, dtype=torch.uint8, device="cuda")
    assert lib.pe_set_workspace(h, P(tiny), tiny.numel()) == B.PE_OK
    assert load() == B.PE_ERR_NOMEM
    info = (ctypes.c_size_t * 4)()
    assert lib.pe_workspace_info(h, info) == B.PE_OK
    assert info[3] > tiny.numel()
    # the estimated size suffices
    assert lib.pe_workspace_size(h, s.n_bead, s.n_body, s.n_ion, ctypes.byref(nbytes)) == B.PE_OK
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    assert lib.pe_set_workspace(h, P(ws), ws.numel()) == B.PE_OK
    del tiny
    assert load() == B.PE_OK, lib.pe_last_error(h)
    q = torch.empty(s.n_bead, dtype=torch.float64, device="cuda")
    dp = torch.empty(s.n_body, dtype=torch.float64, device="cuda")
    si = B.pe_solve_info()
    assert lib.pe_solve_polarization(h, None, P(q), P(dp), None, ctypes.byref(si)) == B.PE_OK
    np.testing.assert_allclose(q.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert lib.pe_workspace_info(h, info) == B.PE_OK
    assert info[0] == ws.numel() and 0 < info[1] <= info[0] and info[2] <= info[0]
    # move everything into a larger region, release the old one, solve again
    ws2 = torch.empty(2 * nbytes.value, dtype=torch.uint8, device="cuda")
    assert lib.pe_set_workspace(h, P(ws2), ws2.numel()) == B.PE_OK
    ws.fill_(0xFF)   # the old region no longer holds anything of the context's
    del ws
    q2 = torch.empty_like(q)
    assert lib.pe_solve_polarization(h, None, P(q2), P(dp), None, ctypes.byref(si)) == B.PE_OK
    np.testing.assert_allclose(q2.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert lib.pe_destroy(h) == B.PE_OK


def test_workspace_grows_with_the_system(gpu_lib):
    """A context that first held a small system takes a much larger one (the
    binding registers a larger region; live buffers move) and keeps its
    trained network across the move."""
    B = gpu_lib
    small = _system()
    p = B.make_params(small.box, small.mesh, P=8, split_tol=1e-8, precision=B.PE_MIXED)
    ctx = B.Context(p).load(small)
    ctx.pe_guess_init(3)
    w0, _, _ = ctx.pe_guess_debug()
    size0 = ctx.pe_workspace_info()["size"]
    big = inputs.small_random_system(42, n_body=8, level=2, n_ion=3000, L=7.0, sigma=0.1, mesh=(32, 32, 32))
    ctx.load(big)
    assert ctx.pe_workspace_info()["size"] > size0
    w1, _, _ = ctx.pe_guess_debug()
    np.testing.assert_array_equal(w0, w1)
    out = ctx.solve()
    assert out["info"]["rel_residual"] <= 1e-6
    ctx.close()
