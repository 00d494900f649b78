"""Grand capacitance tensor and effective permittivity (FP64).
TEST INFRASTRUCTURE ONLY.

Section "Induced Surface Charge Distribution of Polarizable Bodies", the
equation for the rigid-body moments: the charges and dipoles of all bodies
follow from the body potentials and the applied field through

    [Q; S] = Sigma' M^-1 Sigma'^T [Psi - Psi_0; E0],    C = Sigma' M^-1 Sigma'^T,

where Sigma' (4 N_b x N) stacks the summation tensor Sigma (row i: ones on
the beads of body i) over three rows per body that carry the bead
positions relative to the body centre instead of the ones (appendix
"Summation Tensors").  Row order here: body i's charge row is i; its dipole
rows are N_b + 3 i + d (d = x, y, z), so the field part of the right-hand
vector is E0 repeated for every body.

Section "Cubic array of spheres in an electric field": with neutral bodies
(Q = 0) the potentials follow as Psi - Psi_0 = -C_qPsi^-1 C_qE E0, so the
dipoles are S = (C_SE - C_SPsi C_qPsi^-1 C_qE) E0 and the mean polarization
per volume gives

    eps_eff = eps I + (1/V) sum_{i,j} [C_SE - C_SPsi C_qPsi^-1 C_qE]_{ij}

(the paper's expression eps_f - n < C_SPsi C_qPsi^-1 C_qE - C_SE >, n = N_b/V,
the average taken over the bodies, written per 3 x 3 block).  With the
k = 0 mode of the periodic sum removed, E0 is the mean field, so this is
the effective permittivity of the periodic suspension.

Any dense potential tensor may be passed in: the periodic Ewald one
(oracle.ewald), the free-space one (oracle.freespace) or mode B's discrete
one (oracle.se).
"""
from __future__ import annotations

import numpy as np

from .saddle import body_index, relative_positions


def summation_tensor(body_offsets, bead_pos, body_center):
    """Sigma' (4 n_body x n_bead)."""
    off = np.asarray(body_offsets, dtype=np.int64)
    nb = len(off) - 1
    r = relative_positions(bead_pos, body_center, off)
    Sp = np.zeros((4 * nb, off[-1]))
    for i in range(nb):
        Sp[i, off[i]:off[i + 1]] = 1.0
        for d in range(3):
            Sp[nb + 3 * i + d, off[i]:off[i + 1]] = r[off[i]:off[i + 1], d]
    return Sp


def grand_capacitance(M, body_offsets, bead_pos, body_center):
    """C = Sigma' M^-1 Sigma'^T (4 n_body x 4 n_body) by a dense solve."""
    Sp = summation_tensor(body_offsets, bead_pos, body_center)
    X = np.linalg.solve(M, Sp.T)
    return Sp @ X


def blocks(C, n_body):
    nb = n_body
    return C[:nb, :nb], C[:nb, nb:], C[nb:, :nb], C[nb:, nb:]


def effective_permittivity(C, n_body, volume, eps=1.0):
    """3 x 3 effective permittivity of neutral bodies in the mean field."""
    CqP, CqE, CSP, CSE = blocks(C, n_body)
    D = CSE - CSP @ np.linalg.solve(CqP, CqE)
    T = D.reshape(n_body, 3, n_body, 3).sum(axis=(0, 2))
    return eps * np.eye(3) + T / volume


def moments(C, n_body, dpsi, E0_per_body):
    """[Q; S] = C [dPsi; E0] with E0 given per body (n_body x 3)."""
    v = np.concatenate([np.asarray(dpsi, dtype=np.float64), np.asarray(E0_per_body, dtype=np.float64).reshape(-1)])
    out = C @ v
    return out[:n_body], out[n_body:].reshape(n_body, 3)
