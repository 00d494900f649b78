"""Pins of the paper's own split for shells (section "Spectrally-accurate
Ewald summation": j0^2(ka) in both parts; section "Real-space sum": the
closed form of the real-space kernel and its self term) against the
numerical inverse transform, finite differences, the other split's M, and
mode B's convergence to the exact operator."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import ewald, se
from paper_2401_04865_amd import inputs


def _inverse_transform(r, a, xi):
    """(1/(2 pi^2)) int_0^inf (1 - exp(-k^2/4 xi^2)) j0(ka)^2 sin(kr)/(kr) dk."""
    def f(k):
        if k == 0:
            return 0.0
        j0 = math.sin(k * a) / (k * a)
        return (-math.expm1(-k * k / (4 * xi * xi))) * j0 * j0 * math.sin(k * r) / (k * r)
    step = math.pi / (2 * (r + 2 * a))
    kmax = 6000.0
    edges = np.arange(0.0, kmax + step, step)
    tot = sum(quad(f, lo, hi, limit=100, epsabs=1e-15, epsrel=1e-13)[0] for lo, hi in zip(edges[:-1], edges[1:]))
    # tail beyond kmax: j0^2 averages to 1/(2 (ka)^2), times sin(kr)/(kr)
    # oscillating: below 1/(a^2 r kmax^2)/(2 pi^2) ~ 1e-9 of the value here
    return tot / (2 * math.pi ** 2)


@pytest.mark.parametrize("r", [0.05, 0.2, 0.45, 0.59, 0.61, 0.9, 1.4, 2.0])
def test_real_kernel_is_the_inverse_transform(r):
    a, xi = 0.3, 1.7
    prof = ewald.ShellPaperSplit(a)
    want = _inverse_transform(r, a, xi)
    got = float(prof.real(np.array([r]), None, xi)[0])
    assert abs(got - want) <= 1e-8 * max(abs(want), 1e-3), (got, want)


def test_printed_heaviside_sign_fails_the_transform():
    """The term as printed (both parts with a minus sign) misses the inverse
    transform inside r < 2a: the reading is forced."""
    a, xi, r = 0.3, 1.7, 0.2
    prof = ewald.ShellPaperSplit(a)
    fixed = float(prof.real(np.array([r]), None, xi)[0])
    printed = fixed + 2 * (4 * a - r) / (16 * math.pi * a * a)
    want = _inverse_transform(r, a, xi)
    assert abs(printed - want) > 1e-2 * abs(want)


def test_self_term_is_the_zero_distance_limit():
    """The printed self term is R(0); near zero R falls linearly with slope
    -1/(16 pi a^2) (the j0^2/k^4 tail of the transform: the overlap of two
    shells of radius a is not smooth at zero offset)."""
    a, xi = 0.3, 1.7
    prof = ewald.ShellPaperSplit(a)
    R0 = prof.real_self(0.0, xi)
    for r in (1e-5, 1e-4, 1e-3):
        lin = R0 - r / (16 * math.pi * a * a)
        # what is left is of second order in r
        assert abs(float(prof.real(np.array([r]), None, xi)[0]) - lin) <= r * r


@pytest.mark.parametrize("r", [0.1, 0.5, 0.59, 0.61, 0.7, 1.3])
def test_real_kernel_derivative(r):
    a, xi = 0.3, 1.7
    prof = ewald.ShellPaperSplit(a)
    h = 1e-5
    fd = (prof.real(np.array([r + h]), None, xi) - prof.real(np.array([r - h]), None, xi))[0] / (2 * h)
    d = float(prof.real_deriv(np.array([r]), None, xi)[0])
    assert abs(d - fd) <= 1e-7 * max(abs(fd), 1e-2)


@pytest.mark.parametrize("xi", [1.1, 1.9])
def test_paper_split_gives_the_same_potential_tensor(xi):
    """Both placements of the regularization sum to the same M."""
    s = inputs.small_random_system(3, n_body=2, level=1, n_ion=0, L=6.0, mesh=(32, 32, 32))
    a = 0.12
    M1 = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, xi, profile=ewald.Shell(a))
    M2 = ewald.potential_matrix(s.bead_pos, s.bead_sigma, s.box, xi, profile=ewald.ShellPaperSplit(a))
    assert np.abs(M1 - M2).max() <= 1e-11 * np.abs(M1).max()


def test_modeB_paper_split_converges_with_support():
    s = inputs.small_random_system(4, n_body=1, level=1, n_ion=0, L=5.0, mesh=(24, 24, 24))
    a = 0.15
    prof = ewald.ShellPaperSplit(a)
    pos, sig = s.bead_pos, s.bead_sigma
    xi = 1.4
    M = ewald.potential_matrix(pos, sig, s.box, xi, profile=prof)
    q = np.random.default_rng(0).standard_normal(len(pos))
    want = M @ q
    lt = math.sqrt(math.log(1e14))
    errs = []
    for P, c in ((6, 1.0), (10, 0.95), (14, 0.95)):
        h = s.box[0] / 24
        eta = se.eta_of(h, xi, P, c)
        phi, _ = se.apply(pos, sig, pos, sig, q, s.box, s.mesh, P, xi, eta, 2 * a + lt / xi, profile=prof, same=True)
        errs.append(np.abs(phi - want).max() / np.abs(want).max())
    print(errs)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-7


def test_paper_mode_sphere_dipole_trend():
    """Section "Single sphere in an electric field": an icosphere of N beads,
    each a shell of radius half the bead spacing, in free space: the dipole
    exceeds the conducting sphere's 4 pi eps a_b^3 E0 (the body acts larger
    than a_b) by a relative amount that falls like N^-1/2, about 5 % near
    N = 1000."""
    errs, ns = [], []
    for level in (1, 2, 3, 4):
        pos = inputs.icosphere(level, 1.0)
        n = len(pos)
        a = 0.5 * inputs.min_bead_spacing(pos)
        prof = ewald.Shell(a)
        d = pos[:, None, :] - pos[None, :, :]
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        M = prof.free(r)
        A = np.block([[-M, np.ones((n, 1))], [np.ones((1, n)), np.zeros((1, 1))]])
        b = np.concatenate([-pos[:, 2], [0.0]])
        q = np.linalg.solve(A, b)[:n]
        S = pos[:, 2] @ q
        errs.append(S / (4 * math.pi) - 1.0)
        ns.append(n)
    print(ns, errs)
    assert all(e > 0 for e in errs)
    slope = np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert -0.6 < slope < -0.4
    at1000 = math.exp(np.polyval(np.polyfit(np.log(ns), np.log(errs), 1), math.log(1000)))
    assert 0.03 < at1000 < 0.08
