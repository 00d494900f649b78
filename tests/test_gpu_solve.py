"""Parity of the HIP polarization solve and force pass with the CPU oracle.

The GPU solves the saddle-point system with the discrete spectral-Ewald
operator; the oracle solves it densely (LU) both with that same discrete
operator (mode B, agreement to rounding and solver tolerance) and with the
exact operator (agreement within the discretization error).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import ewald, saddle, se
from paper_2401_04865_amd import inputs

pytestmark = pytest.mark.gpu


def _modeB_dense_solve(s, d, P):
    """Dense solve of the saddle system with the discrete operator."""
    M = se.matrix(s.bead_pos, s.bead_sigma, s.box, s.mesh, P, d["xi"], d["eta"], d["r_cut"])
    A = saddle.saddle_matrix(M, s.body_offsets)
    # right-hand side with the discrete operator for the ion potential
    r = saddle.relative_positions(s.bead_pos, s.body_center, s.body_offsets)
    top = -(r @ s.E0)
    if s.n_ion:
        phi, _ = se.apply(s.bead_pos, s.bead_sigma, s.ion_pos, s.ion_sigma, s.ion_charge, s.box, s.mesh, P,
                          d["xi"], d["eta"], d["r_cut"])
        top = top + phi
    b = np.concatenate([top, s.body_charge])
    x = np.linalg.solve(A, b)
    return x[:s.n_bead], x[s.n_bead:], M


def _modeB_forces(s, q, d, P):
    pos, sig, chg = saddle.all_particles(s, q)
    phi, E = se.apply(pos, sig, pos, sig, chg, s.box, s.mesh, P, d["xi"], d["eta"], d["r_cut"],
                      want_field=True, same=True)
    f = chg[:, None] * (s.E0 + E)
    bi = saddle.body_index(s.body_offsets)
    r = saddle.relative_positions(s.bead_pos, s.body_center, s.body_offsets)
    F = np.zeros((s.n_body, 3))
    L = np.zeros((s.n_body, 3))
    np.add.at(F, bi, f[:s.n_bead])
    np.add.at(L, bi, np.cross(r, f[:s.n_bead]))
    U = 0.5 * chg @ phi - chg @ (pos @ s.E0)
    return F, L, f[s.n_bead:], U


def _continuum_dipole(R, sigma, L):
    def j1(x):
        return math.sin(x) / x ** 2 - math.cos(x) / x if x > 1e-6 else x / 3
    edges = np.arange(0.0, 9.0 / sigma + 2.0, 2.0)
    I = sum(quad(lambda k: math.exp(-sigma ** 2 * k ** 2) * j1(k * R) ** 2, lo, hi)[0]
            for lo, hi in zip(edges[:-1], edges[1:]))
    a = 4 * math.pi * R ** 4 / (3 * (2 * R ** 2 / math.pi * I))
    return a / (1 - a / (3 * L ** 3))


def test_cfg1_solve(gpu_lib):
    """One conducting sphere, 162 beads, sigma 0.2, L = 20, mesh 32, P = 8."""
    s = inputs.config(1)
    # residual 1e-14: with cond ~ 4e4 the charges are then accurate to ~1e-10
    p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-14, max_iters=3000)
    ctx = gpu_lib.Context(p).load(s)
    d = ctx.pe_get_derived()
    out = ctx.solve(check=False)
    q = out["q"].cpu().numpy()
    S = out["dipole"].cpu().numpy()[0]
    info = out["info"]
    print(d, info["iters"], info["rel_residual"])
    assert info["rel_residual"] < 1e-13
    # discrete operator, dense: rounding-level parity
    qb, dpb, _ = _modeB_dense_solve(s, d, 8)
    assert np.abs(q - qb).max() <= 1e-9 * np.abs(qb).max()
    # exact operator, dense: within the spectral-Ewald error at P = 8
    qe, dpe, _, _ = saddle.solve(s, xi=0.6)
    Se = saddle.dipoles(s, qe)[0]
    assert np.abs(S - Se).max() / abs(Se[2]) < 2e-5
    # closed form (continuum conductor + Lorentz field of the images)
    want = _continuum_dipole(1.0, 0.2, 20.0)
    assert abs(S[2] - want) / want < 2e-5
    assert abs(S[0]) < 1e-9 * abs(S[2]) and abs(S[1]) < 1e-9 * abs(S[2])
    ctx.close()


def _charged_small(seed=11):
    return inputs.small_random_system(seed, n_body=3, level=1, n_ion=24, L=7.0, sigma=0.16, mesh=(32, 32, 32),
                                      charges=[0.6, -0.2, 0.0])


def test_solve_and_forces_match_discrete_oracle(gpu_lib):
    """Charged bodies and ions: q, dPsi, body forces/torques/energy and ion
    forces equal the dense discrete-operator oracle."""
    s = _charged_small()
    p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-13)
    ctx = gpu_lib.Context(p).load(s)
    d = ctx.pe_get_derived()
    out = ctx.solve()
    assert out["info"]["rel_residual"] < 1e-12
    f = ctx.forces()
    qb, dpb, _ = _modeB_dense_solve(s, d, 8)
    q = out["q"].cpu().numpy()
    assert np.abs(q - qb).max() <= 1e-9 * np.abs(qb).max()
    F, L, fi, U = _modeB_forces(s, qb, d, 8)
    Fg = f["body_force"].cpu().numpy()
    Lg = f["body_torque"].cpu().numpy()
    fig = f["ion_force"].cpu().numpy()
    assert np.abs(Fg - F).max() <= 1e-8 * np.abs(F).max()
    assert np.abs(Lg - L).max() <= 1e-8 * np.abs(L).max()
    assert np.abs(fig - fi).max() <= 1e-8 * np.abs(fi).max()
    assert abs(f["total_energy"] - U) <= 1e-9 * abs(U)
    # body charges hold exactly
    bi = saddle.body_index(s.body_offsets)
    np.testing.assert_allclose(np.bincount(bi, q), s.body_charge, atol=1e-12)
    ctx.close()


def test_solve_and_forces_converge_to_exact_oracle(gpu_lib):
    """Tight discretization (P = 14, eta_c = 0.95, split 1e-12): the GPU
    agrees with the exact dense oracle to about 1e-8."""
    s = _charged_small(12)
    s.mesh = (48, 48, 48)
    p = gpu_lib.make_params(s.box, s.mesh, P=14, eta_c=0.95, split_tol=1e-12, rel_tol=1e-13)
    ctx = gpu_lib.Context(p).load(s)
    out = ctx.solve()
    f = ctx.forces()
    qe, dpe, M, b = saddle.solve(s, xi=1.1)
    ref = saddle.forces_torques(s, qe, 1.1)
    q = out["q"].cpu().numpy()
    assert np.abs(q - qe).max() <= 2e-8 * np.abs(qe).max()
    Fg = f["body_force"].cpu().numpy()
    assert np.abs(Fg - ref["body_force"]).max() <= 1e-7 * np.abs(ref["body_force"]).max()
    # torques are sums of r x f with large cancellation: scale by bead forces
    Lg = f["body_torque"].cpu().numpy()
    r = saddle.relative_positions(s.bead_pos, s.body_center, s.body_offsets)
    scale = np.abs(ref["bead_force"]).max() * np.abs(r).max()
    assert np.abs(Lg - ref["body_torque"]).max() <= 1e-7 * scale
    assert abs(f["total_energy"] - ref["total_energy"]) <= 1e-8 * abs(ref["total_energy"])
    # momentum balance: sum of all forces = Q_tot E0
    tot = Fg.sum(0) + f["ion_force"].cpu().numpy().sum(0)
    Qt = s.body_charge.sum() + s.ion_charge.sum()
    np.testing.assert_allclose(tot, Qt * s.E0, atol=1e-7 * np.abs(Fg).max())
    ctx.close()


def test_mixed_precision_solve(gpu_lib):
    """Float operator inside double refinement reaches the double residual
    target; the charges agree with the double solve to the float bound."""
    s = _charged_small(13)
    res = {}
    for prec in (gpu_lib.PE_FP64, gpu_lib.PE_MIXED):
        p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-10, precision=prec)
        ctx = gpu_lib.Context(p).load(s)
        out = ctx.solve()
        res[prec] = (out["q"].cpu().numpy(), out["info"], ctx.forces())
        ctx.close()
    q64, i64, f64 = res[gpu_lib.PE_FP64]
    q32, i32, f32 = res[gpu_lib.PE_MIXED]
    print(i64["iters"], i32["iters"], i32["outer_refinements"], i32["rel_residual"])
    assert i32["rel_residual"] <= 1e-10
    assert i32["matvecs_fp32"] > 0 and i32["outer_refinements"] >= 1
    assert np.linalg.norm(q32 - q64) <= 1e-6 * np.linalg.norm(q64)
    F64, F32 = f64["body_force"].cpu().numpy(), f32["body_force"].cpu().numpy()
    rms = np.sqrt((F64 ** 2).mean())
    assert np.abs(F32 - F64).max() <= 1e-4 * rms


def test_no_ions_solve_and_forces(gpu_lib):
    """Charged bodies with no ions (empty ion sets): in double the charges,
    body forces, torques and energy equal the dense discrete-operator oracle;
    the mixed path reaches its residual target and agrees to the float bound."""
    s = inputs.small_random_system(31, n_body=3, level=1, n_ion=0, L=7.0, sigma=0.16, mesh=(32, 32, 32),
                                   charges=[0.6, -0.2, 0.0])
    assert s.n_ion == 0
    res = {}
    for prec, tol in ((gpu_lib.PE_FP64, 1e-13), (gpu_lib.PE_MIXED, 1e-10)):
        p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=tol, precision=prec)
        ctx = gpu_lib.Context(p).load(s)
        d = ctx.pe_get_derived()
        out = ctx.solve()
        f = ctx.forces()
        res[prec] = (out["q"].cpu().numpy(), out["info"], f["body_force"].cpu().numpy(),
                     f["body_torque"].cpu().numpy(), f["total_energy"], d)
        ctx.close()
    q64, i64, F64, L64, U64, d = res[gpu_lib.PE_FP64]
    assert i64["rel_residual"] < 1e-12
    qb, _, _ = _modeB_dense_solve(s, d, 8)
    assert np.abs(q64 - qb).max() <= 1e-9 * np.abs(qb).max()
    F, L, fi, U = _modeB_forces(s, qb, d, 8)
    assert fi.shape == (0, 3)
    assert np.abs(F64 - F).max() <= 1e-8 * np.abs(F).max()
    assert np.abs(L64 - L).max() <= 1e-8 * np.abs(L).max()
    assert abs(U64 - U) <= 1e-9 * abs(U)
    q32, i32, F32, _, _, _ = res[gpu_lib.PE_MIXED]
    print(i64["iters"], i32["iters"], i32["rel_residual"])
    assert i32["rel_residual"] <= 1e-10
    assert np.linalg.norm(q32 - q64) <= 1e-6 * np.linalg.norm(q64)
    assert np.abs(F32 - F).max() <= 1e-4 * np.sqrt((F ** 2).mean())


def test_saddle_operator_matches_discrete_matrix(gpu_lib):
    """pe_apply_saddle equals the dense discrete saddle matrix times x."""
    import torch
    s = _charged_small(14)
    p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8)
    ctx = gpu_lib.Context(p).load(s)
    d = ctx.pe_get_derived()
    M = se.matrix(s.bead_pos, s.bead_sigma, s.box, s.mesh, 8, d["xi"], d["eta"], d["r_cut"])
    A = saddle.saddle_matrix(M, s.body_offsets)
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    ctx.pe_apply_saddle(torch.as_tensor(x, device="cuda"), y)
    np.testing.assert_allclose(y.cpu().numpy(), A @ x, atol=1e-11 * np.abs(A @ x).max())
    ctx.close()


def test_error_paths(gpu_lib):
    import torch
    B = gpu_lib
    s = _charged_small(15)
    p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-14, max_iters=2)
    ctx = B.Context(p)
    q = torch.zeros(s.n_bead, dtype=torch.float64, device="cuda")
    dp = torch.zeros(s.n_body, dtype=torch.float64, device="cuda")
    st, _ = ctx.pe_solve_polarization(None, q, dp, check=False)
    assert st == B.PE_ERR_STATE
    ctx.load(s)
    out = ctx.solve(check=False)
    assert out["status"] == B.PE_ERR_NOT_CONVERGED
    assert out["info"]["iters"] == 2
    # r_cut beyond half the box is rejected before any launch
    p2 = B.make_params(s.box, s.mesh, P=8, r_cut=4.0)
    ctx2 = B.Context(p2)
    with pytest.raises(B.PEError):
        ctx2.load(s)
    bad = inputs.small_random_system(15, n_body=1, level=1, n_ion=2, L=7.0, mesh=(32, 32, 32))
    bad.bead_pos[3, 1] = np.nan
    with pytest.raises(B.PEError):
        ctx2.load(bad)
    ctx.close()
    ctx2.close()


def test_cfg2_full_size(gpu_lib):
    """Two 642-bead spheres 2.5 apart + 2000 ions, mesh 64: double and mixed
    solves reach 1e-6 with the double operator; sampled potentials of seeded
    charges agree with the exact oracle within the discretization error."""
    import torch
    s = inputs.config(2)
    infos = {}
    for prec in (gpu_lib.PE_FP64, gpu_lib.PE_MIXED):
        p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8, precision=prec)
        ctx = gpu_lib.Context(p).load(s)
        out = ctx.solve()
        f = ctx.forces()
        infos[prec] = (out, f)
        q = out["q"].cpu().numpy()
        bi = saddle.body_index(s.body_offsets)
        # the constraint rows are part of the residual: |sum q - Q| <= ||b - A x||
        res = out["info"]["rel_residual"] * out["info"]["rhs_norm"]
        assert np.abs(np.bincount(bi, q) - s.body_charge).max() <= res
        assert out["info"]["rel_residual"] <= 1e-6
        if prec == gpu_lib.PE_FP64:
            rng = np.random.default_rng(2)
            chg = np.concatenate([rng.standard_normal(s.n_bead) * 0.1, s.ion_charge])
            psi, E = ctx.apply(torch.as_tensor(chg, device="cuda"), field=True)
            pos, sig, _ = saddle.all_particles(s, np.zeros(s.n_bead))
            smp = np.concatenate([rng.choice(s.n_bead, 12, replace=False),
                                  s.n_bead + rng.choice(s.n_ion, 12, replace=False)])
            ex, Eex = ewald.potential_field(pos[smp], sig[smp], pos, sig, chg, s.box, 0.5)
            psi = psi.cpu().numpy()[smp]
            E = E.cpu().numpy()[smp]
            assert np.abs(psi - ex).max() <= 1e-4 * np.abs(ex).max()
            assert np.abs(E - Eex).max() <= 2e-3 * np.abs(Eex).max()
        ctx.close()
    (o64, f64), (o32, f32) = infos[gpu_lib.PE_FP64], infos[gpu_lib.PE_MIXED]
    S64, S32 = o64["dipole"].cpu().numpy(), o32["dipole"].cpu().numpy()
    print("cfg2 iters", o64["info"]["iters"], o32["info"]["iters"], "S", S64)
    # both solves at residual 1e-6: dipoles agree to the solve tolerance
    assert np.abs(S64 - S32).max() <= 1e-4 * np.abs(S64).max()


def test_block_preconditioner_same_solution_fewer_iterations(gpu_lib):
    """Flexible GMRES with the per-body block preconditioner reaches the same
    charges as the plain solve (to the solve tolerance) in fewer iterations,
    in double and in mixed precision."""
    s = inputs.small_random_system(21, n_body=4, level=2, n_ion=40, L=8.0, sigma=0.1, mesh=(40, 40, 40),
                                   charges=[0.5, 0.0, -0.3, 0.1])
    out = {}
    for pre in (0, 1):
        for prec in (gpu_lib.PE_FP64, gpu_lib.PE_MIXED):
            p = gpu_lib.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-10, precond=pre, precision=prec)
            ctx = gpu_lib.Context(p).load(s)
            r = ctx.solve()
            out[(pre, prec)] = (r["q"].cpu().numpy(), r["info"])
            ctx.close()
    q0, i0 = out[(0, gpu_lib.PE_FP64)]
    for key, (q, info) in out.items():
        assert info["rel_residual"] <= 1e-10
        # mixed precision forms the right-hand side (ion potential at the
        # beads) in single precision like every other sum, so it solves a
        # system whose data differ at the float level: the float bound
        bound = 1e-7 if key[1] == gpu_lib.PE_FP64 else 2e-6
        assert np.linalg.norm(q - q0) <= bound * np.linalg.norm(q0), key
    print({k: v[1]["iters"] for k, v in out.items()})
    assert out[(1, gpu_lib.PE_FP64)][1]["iters"] < 0.5 * i0["iters"]
