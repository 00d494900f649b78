"""Grand capacitance tensor and effective permittivity on the GPU against
the oracle: the dense C = Sigma' M^-1 Sigma'^T of the same discrete
operator (mode B; rounding and solver tolerance only), of the exact
potential tensor (within the spectral-Ewald discretization error), and the
closed form of the periodic conducting sphere."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import capacitance, ewald, se
from paper_2401_04865_amd import inputs

pytestmark = pytest.mark.gpu


def _small():
    return inputs.small_random_system(51, n_body=3, level=1, n_ion=10, L=7.0, sigma=0.16, mesh=(32, 32, 32),
                                      charges=[0.0, 0.0, 0.0])


@pytest.mark.parametrize("precond", [1, 0])
def test_capacitance_matches_discrete_oracle(gpu_lib, precond):
    B = gpu_lib
    s = _small()
    p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-12, precond=precond)
    ctx = B.Context(p).load(s)
    d = ctx.pe_get_derived()
    C, eps, info = ctx.capacitance()
    C = C.cpu().numpy()
    print(precond, info["iters"], info["matvecs_fp64"], info["rel_residual"])
    assert info["rel_residual"] <= 1e-12
    M = se.matrix(s.bead_pos, s.bead_sigma, s.box, s.mesh, 8, d["xi"], d["eta"], d["r_cut"])
    Cb = capacitance.grand_capacitance(M, s.body_offsets, s.bead_pos, s.body_center)
    assert np.abs(C - Cb).max() <= 1e-9 * np.abs(Cb).max()
    eb = capacitance.effective_permittivity(Cb, s.n_body, float(np.prod(s.box)))
    assert np.abs(eps - eb).max() <= 1e-9 * abs(eb[0, 0] - 1)
    # the exact tensor: within the discretization error at P = 8
    Me = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, 1.0)
    Ce = capacitance.grand_capacitance(Me, s.body_offsets, s.bead_pos, s.body_center)
    assert np.abs(C - Ce).max() <= 1e-4 * np.abs(Ce).max()
    ctx.close()


def test_preconditioner_cuts_iterations(gpu_lib):
    B = gpu_lib
    s = _small()
    its = {}
    for pre in (0, 1):
        p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-10, precond=pre)
        ctx = B.Context(p).load(s)
        its[pre] = ctx.capacitance(want_C=False)[2]["iters"]
        ctx.close()
    print(its)
    assert its[1] < its[0]


def test_periodic_sphere_permittivity(gpu_lib):
    """One 162-bead sphere (sigma 0.2, L = 20, mesh 32): eps_eff = 1 +
    alpha' / V with the Lorentz-corrected polarizability of the continuum
    Gaussian-smeared conducting sphere, isotropic."""
    B = gpu_lib
    s = inputs.config(1)
    p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-12)
    ctx = B.Context(p).load(s)
    C, eps, info = ctx.capacitance()

    def j1(x):
        return math.sin(x) / x ** 2 - math.cos(x) / x if x > 1e-6 else x / 3
    edges = np.arange(0.0, 9.0 / 0.2 + 2.0, 1.0)
    I = sum(quad(lambda k: math.exp(-0.04 * k * k) * j1(k) ** 2, lo, hi, limit=200)[0]
            for lo, hi in zip(edges[:-1], edges[1:]))
    alpha = 4 * math.pi / (3 * (2 / math.pi) * I)
    V = 20.0 ** 3
    want = 1 + alpha / (1 - alpha / (3 * V)) / V
    print(eps, want, info["iters"])
    assert abs(eps[2, 2] - want) <= 2e-5 * (want - 1)
    assert np.abs(np.diag(eps) - eps[2, 2]).max() <= 1e-9 * (want - 1)
    assert np.abs(eps - np.diag(np.diag(eps))).max() <= 1e-9 * (want - 1)
    Cn = C.cpu().numpy()
    np.testing.assert_allclose(Cn, Cn.T, atol=1e-9 * np.abs(Cn).max())
    ctx.close()


def test_cubic_lattice_couplings_vanish(gpu_lib):
    """A 2 x 2 x 2 simple-cubic lattice of 42-bead spheres: the charge-field
    and dipole-potential couplings vanish and the permittivity is isotropic
    (to the discretization's symmetry breaking, which the mesh keeps small)."""
    B = gpu_lib
    s = inputs.config(3, nside=2, level=1, n_ion=0, sigma=0.2, mesh=(32, 32, 32))
    p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-8, rel_tol=1e-12)
    ctx = B.Context(p).load(s)
    C, eps, info = ctx.capacitance()
    C = C.cpu().numpy()
    nb = s.n_body
    CqP, CqE, CSP = C[:nb, :nb], C[:nb, nb:], C[nb:, :nb]
    print(eps, np.abs(CqE).max() / np.abs(CqP).max())
    assert np.abs(CqE).max() <= 1e-6 * np.abs(CqP).max()
    assert np.abs(CSP).max() <= 1e-6 * np.abs(CqP).max()
    np.testing.assert_allclose(np.diag(eps), eps[0, 0], rtol=1e-6)
    Me = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, 1.0)
    Ce = capacitance.grand_capacitance(Me, s.body_offsets, s.bead_pos, s.body_center)
    ee = capacitance.effective_permittivity(Ce, nb, float(np.prod(s.box)))
    assert abs(eps[0, 0] - ee[0, 0]) <= 1e-4 * (ee[0, 0] - 1)
    ctx.close()
