"""Mode B: the discretized spectral-Ewald operator, written out by brute force.
TEST INFRASTRUCTURE ONLY.

This reproduces, with no FFT, no sorting and no neighbour lists, the discrete
operator that a spectral-Ewald implementation evaluates (section
"Spectrally-accurate Ewald summation": wave-space split of Lindbo and
Tornberg, spreading, scaling, Parseval contraction by the trapezoid rule;
section "Spectral Ewald implementation", steps 1-6).  It pins an
implementation's *discretization* to rounding level, separately from the
method's truncation error, which the Ewald module pins.

With grid spacing h = L/N per axis, grid points x_m = m h (m = 0..N-1), the
Gaussian window with the normalisation of a unit Gaussian of per-axis
variance eta/(4 xi^2) (the printed prefactor is garbled; this is the only
normalisation whose transform is exp(-eta k^2 / 8 xi^2)):

    w(d)   = (2 xi^2 / (pi eta))^{3/2} exp(-2 xi^2 |d|^2 / eta)
    H_m    = sum_b q_b w(x_m - x_b)           over the P^3 support of b
    Hh_k   = h^3 sum_m H_m exp(-i k.x_m)       (explicit DFT)
    Ht_k   = G_k Hh_k,  G_k = exp(-(1-eta) k^2 / 4 xi^2) / k^2,  G_0 = 0
    Ht_m   = (1/V) sum_k Ht_k exp(+i k.x_m)    (explicit inverse DFT)
    phi_a  = (h^3/eps) sum_m Ht_m w(x_m - x_a)
    E_a    = -(4 xi^2 h^3 / (eps eta)) sum_m Ht_m (x_m - x_a) w(x_m - x_a)

k = 2 pi n / L with n the signed DFT index (n - N for n >= N/2).  Support
(reading of "the closest P grid points"): even P takes m0 - P/2 + 1 .. m0 + P/2
with m0 = floor(x/h); odd P is centred on rint(x/h); indices wrap mod N and
displacements use the unwrapped index.  eta = (h xi)^2 P / (pi c^2), c = 1 in
the paper's choice of eta.

The full discrete operator adds the truncated real-space sum (pairs closer
than r_c, minimum image), the self term and subtracts the k = 0 constant:

    (M q)_a = phi_a + sum_{b, 0<r<r_c} R_ab(r) q_b + R_aa(0) q_a
              - 1/(eps V) sum_b R_hat_ab(0) q_b
"""
from __future__ import annotations

import math

import numpy as np

from . import ewald


def eta_of(h, xi, P, c=1.0):
    return (h * xi) ** 2 * P / (math.pi * c * c)


def support(x, h, N, P):
    """Unwrapped grid indices of the P support points of coordinate x."""
    if P % 2 == 0:
        m0 = math.floor(x / h)
        return np.arange(m0 - P // 2 + 1, m0 + P // 2 + 1)
    m0 = int(np.rint(x / h))
    return np.arange(m0 - (P - 1) // 2, m0 + (P - 1) // 2 + 1)


def _axis_weights(x, h, N, P, xi, eta):
    idx = support(x, h, N, P)
    d = idx * h - x
    w = math.sqrt(2 * xi * xi / (math.pi * eta)) * np.exp(-2 * xi * xi * d * d / eta)
    return idx % N, d, w


def spread(pos, q, box, mesh, P, xi, eta):
    box = np.asarray(box, dtype=np.float64)
    mesh = tuple(int(m) for m in mesh)
    h = box / np.asarray(mesh)
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    H = np.zeros(mesh)
    for b in range(len(pos)):
        ix, _, wx = _axis_weights(pos[b, 0], h[0], mesh[0], P, xi, eta)
        iy, _, wy = _axis_weights(pos[b, 1], h[1], mesh[1], P, xi, eta)
        iz, _, wz = _axis_weights(pos[b, 2], h[2], mesh[2], P, xi, eta)
        H[np.ix_(ix, iy, iz)] += q[b] * np.einsum("i,j,k->ijk", wx, wy, wz)
    return H


def dft_matrix(N, sign):
    m = np.arange(N)
    return np.exp(sign * 2j * math.pi * np.outer(m, m) / N)


def signed_index(N):
    n = np.arange(N)
    return np.where(n < (N + 1) // 2, n, n - N) if N % 2 else np.where(n < N // 2, n, n - N)


def greens(box, mesh, xi, eta, profile=None):
    """G_k, times the profile's wave-space form factor when the split puts
    part of the regularization there (the paper's shell split: j0^2(ka))."""
    box = np.asarray(box, dtype=np.float64)
    ks = [2 * math.pi * signed_index(N) / L for N, L in zip(mesh, box)]
    kk = ks[0][:, None, None] ** 2 + ks[1][None, :, None] ** 2 + ks[2][None, None, :] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.exp(-(1.0 - eta) * kk / (4 * xi * xi)) / kk * ewald._wave_form(profile, kk)
    G[0, 0, 0] = 0.0
    return G


def scaled_grid(H, box, mesh, xi, eta, profile=None):
    """Ht_m from H_m through the explicit forward DFT, scaling and inverse."""
    box = np.asarray(box, dtype=np.float64)
    h = box / np.asarray(mesh)
    h3 = float(np.prod(h))
    V = float(np.prod(box))
    Fx, Fy, Fz = (dft_matrix(N, -1) for N in mesh)
    Hh = h3 * np.einsum("ai,bj,ck,ijk->abc", Fx, Fy, Fz, H, optimize=True)
    Ht_hat = greens(box, mesh, xi, eta, profile) * Hh
    Bx, By, Bz = (dft_matrix(N, +1) for N in mesh)
    Ht = np.einsum("ia,jb,kc,abc->ijk", Bx, By, Bz, Ht_hat, optimize=True) / V
    return Ht.real


def gather(Ht, pos, box, mesh, P, xi, eta, eps=1.0, want_field=False):
    box = np.asarray(box, dtype=np.float64)
    h = box / np.asarray(mesh)
    h3 = float(np.prod(h))
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    phi = np.zeros(len(pos))
    E = np.zeros((len(pos), 3))
    for a in range(len(pos)):
        ix, dx, wx = _axis_weights(pos[a, 0], h[0], mesh[0], P, xi, eta)
        iy, dy, wy = _axis_weights(pos[a, 1], h[1], mesh[1], P, xi, eta)
        iz, dz, wz = _axis_weights(pos[a, 2], h[2], mesh[2], P, xi, eta)
        blk = Ht[np.ix_(ix, iy, iz)]
        W = np.einsum("i,j,k->ijk", wx, wy, wz)
        phi[a] = h3 / eps * np.sum(blk * W)
        if want_field:
            c = -4 * xi * xi * h3 / (eps * eta)
            E[a, 0] = c * np.sum(blk * W * dx[:, None, None])
            E[a, 1] = c * np.sum(blk * W * dy[None, :, None])
            E[a, 2] = c * np.sum(blk * W * dz[None, None, :])
    return phi, E


def wave_potential(pos_t, pos_s, q_s, box, mesh, P, xi, eta, eps=1.0, want_field=False, profile=None):
    H = spread(pos_s, q_s, box, mesh, P, xi, eta)
    Ht = scaled_grid(H, box, mesh, xi, eta, profile)
    return gather(Ht, pos_t, box, mesh, P, xi, eta, eps, want_field)


def real_potential(pos_t, sig_t, pos_s, sig_s, q_s, box, xi, r_c, eps=1.0, profile=None,
                   want_field=False, same=False):
    """Truncated real-space sum over pairs with minimum-image distance < r_c
    (r_c <= L/2, so one image at most), plus the self term when the target
    set is the source set (``same``)."""
    profile = ewald._profile(profile)
    box = np.asarray(box, dtype=np.float64)
    pos_t = np.asarray(pos_t, dtype=np.float64)
    pos_s = np.asarray(pos_s, dtype=np.float64)
    phi = np.zeros(len(pos_t))
    E = np.zeros((len(pos_t), 3))
    for a in range(len(pos_t)):
        d = ewald.min_image(pos_t[a] - pos_s, box)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        m = r < r_c
        if same:
            m[a] = False
        s2 = profile.pair_s2(sig_t[a], sig_s[m])
        phi[a] = np.sum(profile.real(r[m], s2, xi, eps) * q_s[m])
        if want_field:
            dR = profile.real_deriv(r[m], s2, xi, eps)
            E[a] = -np.sum((dR * q_s[m] / r[m])[:, None] * d[m], axis=0)
        if same:
            phi[a] += profile.real_self(profile.pair_s2(sig_t[a], sig_t[a]), xi, eps) * q_s[a]
    return phi, E


def k0_constant(sig_t, sig_s, q_s, box, xi, eps=1.0, profile=None):
    profile = ewald._profile(profile)
    V = float(np.prod(box))
    s2 = profile.pair_s2(np.asarray(sig_t)[:, None], np.asarray(sig_s)[None, :])
    return (profile.rhat0(s2, xi) @ np.asarray(q_s)) / (eps * V)


def apply(pos_t, sig_t, pos_s, sig_s, q_s, box, mesh, P, xi, eta, r_c, eps=1.0,
          profile=None, want_field=False, same=False):
    """Full discrete operator: potential (and field) at the targets."""
    pw, Ew = wave_potential(pos_t, pos_s, q_s, box, mesh, P, xi, eta, eps, want_field, profile)
    pr, Er = real_potential(pos_t, sig_t, pos_s, sig_s, q_s, box, xi, r_c, eps, profile,
                            want_field, same)
    c = k0_constant(sig_t, sig_s, q_s, box, xi, eps, profile)
    return pw + pr - c, Ew + Er


def matrix(pos, sig, box, mesh, P, xi, eta, r_c, eps=1.0, profile=None):
    """Dense discrete operator of one particle set, column by column."""
    n = len(pos)
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j], _ = apply(pos, sig, pos, sig, e, box, mesh, P, xi, eta, r_c, eps, profile,
                           same=True)
    return M
