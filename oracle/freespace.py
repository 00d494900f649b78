"""Free-space (non-periodic) counterparts of the oracle quantities, FP64.
TEST INFRASTRUCTURE ONLY.

Used for closed-form pins that need an isolated body: with no periodic
images the potential tensor of Gaussian charges is M_ab = erf(r/(sqrt2 s)) /
(4 pi eps r), s^2 = sigma_a^2 + sigma_b^2, and M_aa = 2/(sqrt(pi) sqrt2 s)/(4 pi eps)
(the r -> 0 limit).  The saddle system, dipoles and forces are those of the
periodic module (section "Induced Surface Charge Distribution of Polarizable
Bodies"; section "Forces and Torques").
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .saddle import summation_matrix, relative_positions, body_index


def potential_matrix(pos, sig, eps=1.0):
    pos = np.asarray(pos, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    s2 = sig[:, None] ** 2 + sig[None, :] ** 2
    b = 1.0 / np.sqrt(2.0 * s2)
    with np.errstate(divide="ignore", invalid="ignore"):
        M = erf(b * r) / (4 * math.pi * eps * r)
    diag = (2.0 / math.sqrt(math.pi)) * b / (4 * math.pi * eps)
    M[r == 0] = diag[r == 0]
    return M


def field_matrix(pos, sig, eps=1.0):
    """G[a,b,:] = grad_a M_ab (zero on the diagonal)."""
    pos = np.asarray(pos, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    s2 = sig[:, None] ** 2 + sig[None, :] ** 2
    b = 1.0 / np.sqrt(2.0 * s2)
    with np.errstate(divide="ignore", invalid="ignore"):
        dM = ((2 * b / math.sqrt(math.pi)) * np.exp(-(b * r) ** 2) * r - erf(b * r)) / (4 * math.pi * eps * r * r)
        G = (dM / r)[:, :, None] * d
    G[r == 0] = 0.0
    return G


def solve(body_offsets, bead_pos, bead_sigma, body_center, body_charge, E0, eps=1.0):
    M = potential_matrix(bead_pos, bead_sigma, eps)
    S = summation_matrix(body_offsets)
    nb = S.shape[0]
    A = np.block([[-M, S.T], [S, np.zeros((nb, nb))]])
    r = relative_positions(bead_pos, body_center, body_offsets)
    b = np.concatenate([-(r @ E0), body_charge])
    x = np.linalg.solve(A, b)
    n = len(bead_pos)
    return x[:n], x[n:], M


def forces_torques(body_offsets, bead_pos, bead_sigma, body_center, q, E0, eps=1.0):
    G = field_matrix(bead_pos, bead_sigma, eps)
    E = -np.einsum("abk,b->ak", G, q)
    f = q[:, None] * (np.asarray(E0)[None, :] + E)
    r = relative_positions(bead_pos, body_center, body_offsets)
    bi = body_index(body_offsets)
    nb = len(body_offsets) - 1
    F = np.zeros((nb, 3))
    L = np.zeros((nb, 3))
    S = np.zeros((nb, 3))
    np.add.at(F, bi, f)
    np.add.at(L, bi, np.cross(r, f))
    np.add.at(S, bi, r * q[:, None])
    M = potential_matrix(bead_pos, bead_sigma, eps)
    U = 0.5 * q @ (M @ q) - q @ (np.asarray(bead_pos) @ E0)
    return dict(bead_force=f, body_force=F, body_torque=L, dipole=S, energy=float(U))
