"""Conductor saddle-point system, its dense solve and the derived body
quantities (FP64).  TEST INFRASTRUCTURE ONLY.

Section "Induced Surface Charge Distribution of Polarizable Bodies":

* bead potential relative to the applied potential psi_0 = -x.E0 equals the
  body's, plus r.E0:  psi_ij - psi_0(x_ij) = (Psi_i - Psi_0,i) + r_ij.E0,
  r_ij = x_ij - X_i;
* psi - psi_0 = M q over *all* charges (beads and ions), eq. for the bead
  potential in terms of the potential tensor;
* net body charge Q_i = sum_j q_ij.

Ions are single-bead bodies whose one charge is fixed by their own net-charge
constraint, so they are eliminated: their potential M_bead,ion q_ion moves to
the right-hand side.  With dPsi = Psi - Psi_0 the system reads

    [ -M  Sigma^T ] [ q    ]   [ -r.E0 + M_bi q_ion ]
    [ Sigma   0   ] [ dPsi ] = [  Q                 ]

(the saddle-point system of the paper, with the ion term added).  Then

* dipole S_i = sum_j r_ij q_ij                      (eq. for the rigid dipole)
* bead force f_a = q_a E0 - 1/2 (grad_a M) : q q = q_a (E0 + E_a),
  E_a = -sum_{b} grad_a M_ab q_b                    (bead-force equation and
  its appendix derivation; M symmetric, grad_a M_aa = 0)
* F_i = sum_j f_ij,  L_i = sum_j r_ij x f_ij        (body force and torque)
* energy U = 1/2 q.Mq - sum_a q_a x_a.E0 over all charges; per body
  U_i = sum_j (1/2 q_ij (Mq)_ij - q_ij x_ij.E0).  This is the energy whose
  negative gradient is the bead force above (the printed energy lines
  disagree with each other; for neutral bodies this equals the first one).
"""
from __future__ import annotations

import numpy as np

from . import ewald


def body_index(body_offsets):
    off = np.asarray(body_offsets, dtype=np.int64)
    return np.repeat(np.arange(len(off) - 1), np.diff(off))


def summation_matrix(body_offsets):
    """Sigma (n_body x n_bead): row i has ones on the beads of body i."""
    off = np.asarray(body_offsets, dtype=np.int64)
    S = np.zeros((len(off) - 1, off[-1]))
    for i in range(len(off) - 1):
        S[i, off[i]:off[i + 1]] = 1.0
    return S


def relative_positions(bead_pos, body_center, body_offsets):
    return np.asarray(bead_pos) - np.asarray(body_center)[body_index(body_offsets)]


def ion_potential_at_beads(sys, xi, eps=1.0, profile=None):
    if sys.n_ion == 0:
        return np.zeros(sys.n_bead)
    phi, _ = ewald.potential_field(sys.bead_pos, sys.bead_sigma, sys.ion_pos, sys.ion_sigma,
                                   sys.ion_charge, sys.box, xi, eps, profile, want_field=False)
    return phi


def rhs(sys, xi, eps=1.0, profile=None):
    r = relative_positions(sys.bead_pos, sys.body_center, sys.body_offsets)
    top = -(r @ sys.E0) + ion_potential_at_beads(sys, xi, eps, profile)
    return np.concatenate([top, sys.body_charge])


def saddle_matrix(M, body_offsets):
    S = summation_matrix(body_offsets)
    nb = S.shape[0]
    return np.block([[-M, S.T], [S, np.zeros((nb, nb))]])


def solve(sys, xi, eps=1.0, profile=None, M=None):
    """Dense LU solve of the saddle system.  Returns (q, dpsi, M, b)."""
    if M is None:
        M = ewald.potential_matrix(sys.bead_pos, sys.bead_sigma, sys.box, xi, eps, profile)
    A = saddle_matrix(M, sys.body_offsets)
    b = rhs(sys, xi, eps, profile)
    x = np.linalg.solve(A, b)
    return x[:sys.n_bead], x[sys.n_bead:], M, b


def apply_saddle(M, body_offsets, x):
    return saddle_matrix(M, body_offsets) @ x


def dipoles(sys, q):
    r = relative_positions(sys.bead_pos, sys.body_center, sys.body_offsets)
    out = np.zeros((sys.n_body, 3))
    np.add.at(out, body_index(sys.body_offsets), r * q[:, None])
    return out


def all_particles(sys, q):
    pos = np.concatenate([sys.bead_pos, sys.ion_pos], 0)
    sig = np.concatenate([sys.bead_sigma, sys.ion_sigma])
    chg = np.concatenate([q, sys.ion_charge])
    return pos, sig, chg


def forces_torques(sys, q, xi, eps=1.0, profile=None):
    """Bead/ion forces, body forces, torques, energies (see module doc)."""
    pos, sig, chg = all_particles(sys, q)
    phi, E = ewald.potential_field(pos, sig, pos, sig, chg, sys.box, xi, eps, profile,
                                   want_field=True)
    f = chg[:, None] * (sys.E0[None, :] + E)
    u = 0.5 * chg * phi - chg * (pos @ sys.E0)
    nb, n = sys.n_body, sys.n_bead
    bi = body_index(sys.body_offsets)
    r = relative_positions(sys.bead_pos, sys.body_center, sys.body_offsets)
    F = np.zeros((nb, 3))
    L = np.zeros((nb, 3))
    U = np.zeros(nb)
    np.add.at(F, bi, f[:n])
    np.add.at(L, bi, np.cross(r, f[:n]))
    np.add.at(U, bi, u[:n])
    return dict(bead_force=f[:n], ion_force=f[n:], body_force=F, body_torque=L,
                body_energy=U, ion_energy=u[n:], total_energy=float(u.sum()),
                phi=phi, E=E)
