"""Pins of the grand-capacitance oracle (section "Induced Surface Charge
Distribution of Polarizable Bodies", the rigid-body moment equation; section
"Cubic array of spheres in an electric field", the effective permittivity)
against things other than itself: the pinned dense saddle solve, closed
forms of an isolated Gaussian-smeared conducting sphere, the periodic
conductor with its Lorentz image field, and the symmetries of a cubic
lattice."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import capacitance, ewald, freespace, saddle
from paper_2401_04865_amd import inputs


def _radial(sigma, R, j):
    """int_0^inf exp(-sigma^2 k^2) j_l(kR)^2 dk for l = 0 (j0) or 1 (j1)."""
    def jl(x):
        if j == 0:
            return math.sin(x) / x if x > 1e-8 else 1.0
        return math.sin(x) / x ** 2 - math.cos(x) / x if x > 1e-6 else x / 3
    edges = np.arange(0.0, 9.0 / sigma + 2.0, 1.0)
    return sum(quad(lambda k: math.exp(-sigma ** 2 * k ** 2) * jl(k * R) ** 2, lo, hi, limit=200)[0]
               for lo, hi in zip(edges[:-1], edges[1:]))


def test_capacitance_reproduces_the_saddle_solve():
    """[Q; S] = C [dPsi; E0] with dPsi from the dense saddle solve of charged
    bodies (no ions) in a field, for two fields and two sets of charges:
    catches a transposed Sigma', a wrong row order or a sign slip."""
    s = inputs.small_random_system(5, n_body=3, level=1, n_ion=0, L=7.0, sigma=0.16, mesh=(32, 32, 32),
                                   charges=[0.5, -0.3, 0.1])
    xi = 0.9
    M = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, xi)
    C = capacitance.grand_capacitance(M, s.body_offsets, s.bead_pos, s.body_center)
    for E0, Q in (((0.3, -0.7, 0.4), (0.5, -0.3, 0.1)), ((0.0, 0.0, 1.0), (0.0, 0.0, 0.0))):
        s.E0 = np.asarray(E0, dtype=np.float64)
        s.body_charge = np.asarray(Q, dtype=np.float64)
        q, dpsi, _, _ = saddle.solve(s, xi, M=M)
        Qc, Sc = capacitance.moments(C, s.n_body, dpsi, np.tile(s.E0, (s.n_body, 1)))
        np.testing.assert_allclose(Qc, s.body_charge, atol=1e-10)
        np.testing.assert_allclose(Sc, saddle.dipoles(s, q), atol=1e-10 * np.abs(Sc).max())


def test_capacitance_symmetric_positive_definite():
    s = inputs.small_random_system(6, n_body=3, level=1, n_ion=0, L=7.0, sigma=0.16, mesh=(32, 32, 32))
    M = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, 0.9)
    C = capacitance.grand_capacitance(M, s.body_offsets, s.bead_pos, s.body_center)
    np.testing.assert_allclose(C, C.T, atol=1e-12 * np.abs(C).max())
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0


@pytest.mark.parametrize("level,sigma,gap", [(2, 0.2, 2e-4), (3, 0.05, 5e-4)])
def test_isolated_sphere_closed_forms(level, sigma, gap):
    """Free space, one sphere of radius 1: the capacitance of a conducting
    sphere whose surface charge is smeared by Gaussians of width sigma is
    2 pi^2 eps / int exp(-sigma^2 k^2) j0(k)^2 dk (4 pi eps R as sigma -> 0),
    its polarizability 4 pi eps / (3 K1) with K1 = (2/pi) int exp(-sigma^2
    k^2) j1(k)^2 dk (4 pi eps R^3 as sigma -> 0); the charge and dipole
    couplings vanish.  The discrete sphere matches within its bead gap."""
    pos = inputs.icosphere(level, 1.0)
    n = len(pos)
    sig = np.full(n, sigma)
    M = freespace.potential_matrix(pos, sig)
    C = capacitance.grand_capacitance(M, np.array([0, n]), pos, np.zeros((1, 3)))
    CqP, CqE, CSP, CSE = capacitance.blocks(C, 1)
    cap = 2 * math.pi ** 2 / _radial(sigma, 1.0, 0)
    alpha = 4 * math.pi / (3 * (2 / math.pi) * _radial(sigma, 1.0, 1))
    print(CqP[0, 0], cap, CSE[0, 0], alpha)
    assert abs(CqP[0, 0] - cap) <= gap * cap
    np.testing.assert_allclose(np.diag(CSE), alpha, rtol=gap)
    assert np.abs(CqE).max() <= 1e-10 * cap and np.abs(CSE - np.diag(np.diag(CSE))).max() <= 1e-10 * alpha


def test_periodic_sphere_permittivity_lorentz():
    """One 162-bead sphere (sigma 0.2) in a periodic cube of side 20: the
    effective permittivity is eps (1 + alpha' / V) with alpha' the
    polarizability corrected by the Lorentz field of the images,
    alpha / (1 - alpha / (3 eps V)) (the Clausius-Mossotti relation), and
    isotropic."""
    s = inputs.config(1)
    M = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, 0.6)
    C = capacitance.grand_capacitance(M, s.body_offsets, s.bead_pos, s.body_center)
    V = float(np.prod(s.box))
    eps = capacitance.effective_permittivity(C, 1, V)
    alpha = 4 * math.pi / (3 * (2 / math.pi) * _radial(0.2, 1.0, 1))
    want = 1 + alpha / (1 - alpha / (3 * V)) / V
    print(eps, want)
    assert abs(eps[2, 2] - want) <= 2e-5 * (want - 1)
    np.testing.assert_allclose(np.diag(eps), eps[2, 2], rtol=1e-12)
    assert np.abs(eps - np.diag(np.diag(eps))).max() <= 1e-12


def test_cubic_lattice_couplings_vanish_and_isotropic():
    """A 2 x 2 x 2 simple-cubic lattice of 42-bead spheres: every sphere sits
    at a centre of inversion of the periodic lattice and is itself
    inversion-symmetric, so the charge-field and dipole-potential couplings
    vanish (the paper's statement for cubic arrays); the lattice and the
    icosahedral spheres share the coordinate mirrors and the threefold
    diagonal axes, so the permittivity is isotropic."""
    s = inputs.config(3, nside=2, level=1, n_ion=0, sigma=0.2)
    assert s.n_ion == 0 and s.n_body == 8
    M = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, 1.0)
    C = capacitance.grand_capacitance(M, s.body_offsets, s.bead_pos, s.body_center)
    CqP, CqE, CSP, CSE = capacitance.blocks(C, 8)
    assert np.abs(CqE).max() <= 1e-9 * np.abs(CqP).max()
    assert np.abs(CSP).max() <= 1e-9 * np.abs(CqP).max()
    eps = capacitance.effective_permittivity(C, 8, float(np.prod(s.box)))
    print(eps)
    np.testing.assert_allclose(np.diag(eps), eps[0, 0], rtol=1e-9)
    assert np.abs(eps - np.diag(np.diag(eps))).max() <= 1e-9 * (eps[0, 0] - 1)
    # polarizable inclusions raise the permittivity
    assert eps[0, 0] > 1.0
