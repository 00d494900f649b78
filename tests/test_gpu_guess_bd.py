"""Learned initial guess (network on matrix cores) and Brownian-dynamics step
against CPU references.

* gradients of the device backward pass vs the CPU reference backprop (same
  bf16 operand rounding), whose own formulas are pinned by central
  differences on the CPU;
* device features vs features computed by the oracle from the system;
* training on solves of the method lowers the loss and the initial residual,
  and the Krylov solve still reaches the same charges;
* one BD step vs the oracle's step driven by the oracle's own forces, with
  bit-identical counter-based noise.
"""
import os

import numpy as np
import pytest

from oracle import bd, ewald, mlp, saddle
from paper_2401_04865_amd import inputs

pytestmark = pytest.mark.gpu


def _rows(n, seed=0):
    rng = np.random.default_rng(seed)
    rows = np.zeros((n, 11), dtype=np.float32)
    rows[:, :3] = rng.standard_normal((n, 3))
    rows[:, 3:6] = rng.standard_normal((n, 3))
    t = rng.integers(0, 2, n)
    rows[:, 6] = t == 0
    rows[:, 7] = t == 1
    rows[:, 8] = rng.standard_normal(n) * 0.02
    rows[:, 9] = rng.standard_normal(n) * 0.1
    return rows


def _ctx(B, s, **kw):
    opts = dict(P=8, split_tol=1e-8)
    opts.update(kw)
    p = B.make_params(s.box, s.mesh, **opts)
    return B.Context(p).load(s)


@pytest.mark.parametrize("n_rows", [16, 1000, 4099])
def test_guess_gradient_matches_reference_backprop(gpu_lib, n_rows):
    s = inputs.small_random_system(1, n_body=1, level=1, n_ion=4, L=6.0, mesh=(32, 32, 32))
    ctx = _ctx(gpu_lib, s)
    ctx.pe_guess_init(3)
    rows = _rows(n_rows, n_rows)
    ctx.pe_guess_add_rows(rows)
    P = (np.random.default_rng(5).standard_normal(mlp.NPAR) * 0.3).astype(np.float32)
    _, g, loss = ctx.pe_guess_debug(P, n_rows)
    Lr, gr = mlp.loss_grad(P.astype(np.float64), rows.astype(np.float64), bf=True)
    assert abs(loss - Lr) <= 1e-5 * Lr
    assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()
    # each block of the gradient separately (W1, b1, W2, b2, W3, b3)
    for a, b in ((0, mlp.ob1), (mlp.ob1, mlp.oW2), (mlp.oW2, mlp.ob2), (mlp.ob2, mlp.oW3), (mlp.oW3, mlp.ob3),
                 (mlp.ob3, mlp.NPAR)):
        assert np.abs(g[a:b] - gr[a:b]).max() <= 1e-4 * np.abs(gr[a:b]).max() + 1e-12
    # against the plain double-precision backprop (no operand rounding): the
    # matrix-core products round their operands to bfloat16 (unit roundoff
    # 2^-9 = 2e-3), so each block may differ by a few units of it; 1.5e-2 is
    # about eight (the bf16 reference itself differs from double by at most
    # 5e-3 per block on these inputs)
    L64, g64 = mlp.loss_grad(P.astype(np.float64), rows.astype(np.float64), bf=False)
    assert abs(loss - L64) <= 5e-3 * L64
    for a, b in ((0, mlp.ob1), (mlp.ob1, mlp.oW2), (mlp.oW2, mlp.ob2), (mlp.ob2, mlp.oW3), (mlp.oW3, mlp.ob3),
                 (mlp.ob3, mlp.NPAR)):
        assert np.abs(g[a:b] - g64[a:b]).max() <= 1.5e-2 * np.abs(g64[a:b]).max()
    ctx.close()


def _body_frame_features(s, E_ion):
    R = inputs.quat_to_matrix(s.body_quat)
    bi = saddle.body_index(s.body_offsets)
    r = saddle.relative_positions(s.bead_pos, s.body_center, s.body_offsets)
    E = s.E0[None, :] + E_ion
    f = np.zeros((s.n_bead, 9))
    f[:, 0:3] = np.einsum("nji,nj->ni", R[bi], r)
    f[:, 3:6] = np.einsum("nji,nj->ni", R[bi], E)
    f[:, 6] = s.body_type[bi] == 0
    f[:, 7] = s.body_type[bi] == 1
    f[:, 8] = s.body_charge[bi] / np.diff(s.body_offsets)[bi]
    return f


def test_guess_features_match_oracle(gpu_lib):
    s = inputs.small_random_system(2, n_body=2, level=1, n_ion=16, L=7.0, sigma=0.15, mesh=(40, 40, 40),
                                   charges=[0.4, -0.1])
    s.body_type = np.array([0, 1], dtype=np.int32)
    ctx = _ctx(gpu_lib, s, split_tol=1e-10, P=12)
    ctx.pe_guess_init(1)
    ctx.pe_guess_set_types(s.body_type)
    out = ctx.solve()
    ctx.pe_guess_record(out["q"])
    rows = ctx.pe_guess_rows(s.n_bead)
    _, E = ewald.potential_field(s.bead_pos, s.bead_sigma, s.ion_pos, s.ion_sigma, s.ion_charge, s.box, 1.2)
    f = _body_frame_features(s, E)
    np.testing.assert_allclose(rows[:, :9], f, atol=2e-6 * max(1.0, np.abs(f).max()))
    ctx.close()


def _train_systems(n, seed0):
    out = []
    for k in range(n):
        out.append(inputs.small_random_system(seed0 + k, n_body=3, level=2, n_ion=30, L=9.0, sigma=0.09,
                                              mesh=(48, 48, 48), charges=[0.0, 0.5, -0.5]))
    return out


def test_training_lowers_loss_and_initial_residual(gpu_lib, tmp_path):
    B = gpu_lib
    systems = _train_systems(12, 100)
    ctx = _ctx(B, systems[0], rel_tol=1e-8)
    ctx.pe_guess_init(7)
    for s in systems:
        ctx.load(s)
        out = ctx.solve()
        ctx.pe_guess_record(out["q"])
    l0 = ctx.pe_guess_train(1, 512, 1e-3, 1)
    loss = ctx.pe_guess_train(150, 512, 3e-3, 2)
    print("loss", l0, loss)
    assert loss < 0.2 * l0
    path = tmp_path / "w.bin"
    ctx.pe_guess_save(path)
    ctx.close()
    # held-out system: zero guess vs learned guess, same answer
    test = _train_systems(1, 500)[0]
    res = {}
    for learned in (0, 1):
        p = B.make_params(test.box, test.mesh, P=8, split_tol=1e-8, rel_tol=1e-8, use_learned_guess=learned,
                          precond=0)
        c = B.Context(p)
        if learned:
            c.pe_guess_load(path)
        c.load(test)
        out = c.solve()
        res[learned] = (out["q"].cpu().numpy(), out["info"])
        c.close()
    (q0, i0), (q1, i1) = res[0], res[1]
    print("guess residual", i1["rel_residual_guess"], "iters", i0["iters"], i1["iters"])
    assert i1["rel_residual_guess"] < 0.5
    assert i1["rel_residual"] <= 1e-8
    assert np.linalg.norm(q1 - q0) <= 1e-6 * np.linalg.norm(q0)
    assert i1["iters"] <= i0["iters"]


def test_guess_save_load_roundtrip_and_corrupt_file(gpu_lib, tmp_path):
    import torch
    B = gpu_lib
    s = inputs.small_random_system(4, n_body=2, level=1, n_ion=8, L=6.0, mesh=(32, 32, 32), charges=[0.2, 0.0])
    c1 = _ctx(B, s)
    c1.pe_guess_init(11)
    c1.solve()
    q1 = torch.empty(s.n_bead, dtype=torch.float64, device="cuda")
    c1.pe_guess_predict(q1)
    c1.pe_guess_save(tmp_path / "a.bin")
    c2 = _ctx(B, s)
    c2.pe_guess_load(tmp_path / "a.bin")
    c2.solve()
    q2 = torch.empty_like(q1)
    c2.pe_guess_predict(q2)
    assert torch.equal(q1, q2)
    # the projection makes each body carry its net charge
    bi = saddle.body_index(s.body_offsets)
    np.testing.assert_allclose(np.bincount(bi, q1.cpu().numpy()), s.body_charge, atol=1e-12)
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"PEGUESS1" + os.urandom(64))
    with pytest.raises(B.PEError):
        c2.pe_guess_load(bad)
    c1.close()
    c2.close()


def test_bd_step_matches_oracle(gpu_lib):
    import torch
    B = gpu_lib
    s = inputs.small_random_system(6, n_body=2, level=1, n_ion=10, L=7.0, sigma=0.16, mesh=(48, 48, 48),
                                   charges=[0.5, -0.2])
    p = B.make_params(s.box, s.mesh, P=14, eta_c=0.95, split_tol=1e-12, rel_tol=1e-13)
    ctx = B.Context(p).load(s)
    ctx.solve()
    ctx.forces()
    d = ctx.sys_dev
    dt, kT, gamma, seed, step_no = 1e-3, 1.0, 1.0, 12345, 7
    ctx.pe_bd_step(dt, kT, gamma, seed, step_no, d["bead_pos"], d["body_center"], d["body_quat"], d["ion_pos"])
    qe, dpe, M, b = saddle.solve(s, xi=1.1)
    ref = saddle.forces_torques(s, qe, 1.1)
    pos, X, Q, ion = bd.step(s, ref["body_force"], ref["body_torque"], ref["ion_force"], dt, kT, gamma, seed,
                             step_no)
    np.testing.assert_allclose(d["ion_pos"].cpu().numpy(), ion, atol=1e-9)
    np.testing.assert_allclose(d["body_center"].cpu().numpy(), X, atol=1e-9)
    np.testing.assert_allclose(d["body_quat"].cpu().numpy(), Q, atol=1e-9)
    np.testing.assert_allclose(d["bead_pos"].cpu().numpy(), pos, atol=1e-9)
    # the displacement is dominated by the noise: check it is actually there
    assert np.abs(ion - s.ion_pos).max() > 1e-3
    with pytest.raises(B.PEError):   # positions moved: a new configuration must be loaded
        ctx.pe_solve_polarization(None, torch.empty(s.n_bead, dtype=torch.float64, device="cuda"),
                                  torch.empty(s.n_body, dtype=torch.float64, device="cuda"))
    ctx.close()


def test_bd_step_with_hard_spheres_matches_oracle(gpu_lib):
    """The step with the potential-free hard-sphere forces (ions against ions
    and against beads of the bodies) against the oracle's step with its own
    brute-force hard-sphere forces, driven by the oracle's electrostatic
    forces; noise and all."""
    B = gpu_lib
    s = inputs.small_random_system(8, n_body=2, level=1, n_ion=80, L=6.0, sigma=0.16, mesh=(48, 48, 48),
                                   charges=[0.4, -0.1])
    a = 0.2
    fb_hs, fi_hs = bd.hard_sphere_forces(s, a, 1.0, 1e-3)
    assert np.abs(fb_hs).max() > 0 and np.abs(fi_hs).max() > 0   # both kinds of contact occur
    p = B.make_params(s.box, s.mesh, P=14, eta_c=0.95, split_tol=1e-12, rel_tol=1e-13, hs_radius=a)
    ctx = B.Context(p).load(s)
    ctx.solve()
    ctx.forces()
    d = ctx.sys_dev
    dt, kT, gamma, seed, step_no = 1e-3, 1.0, 1.0, 777, 3
    ctx.pe_bd_step(dt, kT, gamma, seed, step_no, d["bead_pos"], d["body_center"], d["body_quat"], d["ion_pos"])
    qe, dpe, M, b = saddle.solve(s, xi=1.1)
    ref = saddle.forces_torques(s, qe, 1.1)
    pos, X, Q, ion = bd.step(s, ref["body_force"], ref["body_torque"], ref["ion_force"], dt, kT, gamma, seed,
                             step_no, hs_radius=a)
    np.testing.assert_allclose(d["ion_pos"].cpu().numpy(), ion, atol=1e-9)
    np.testing.assert_allclose(d["body_center"].cpu().numpy(), X, atol=1e-9)
    np.testing.assert_allclose(d["body_quat"].cpu().numpy(), Q, atol=1e-9)
    np.testing.assert_allclose(d["bead_pos"].cpu().numpy(), pos, atol=1e-9)
    ctx.close()
