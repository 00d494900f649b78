"""Overdamped Brownian-dynamics step and its counter-based noise (FP64).
TEST INFRASTRUCTURE ONLY.

Section "Brownian dynamics simulations of charged and polarizable colloids in
explicit electrolytes": Euler-Maruyama update of the overdamped Langevin
equation with Stokes drag gamma per particle and no hydrodynamic coupling.
Rigid bodies of N beads move freely (free draining): translational drag
N gamma, rotational drag K = gamma sum_j (|r_j|^2 I - r_j r_j^T) about the
centroid; the rigid velocities of the appendix, u = U + Omega x r, move the
beads.  The Brownian rotation uses any C with C C^T = K^{-1} (here the
Cholesky factor).

Noise: Philox-4x32-10, written from its published definition (Salmon et al.,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011): 10 rounds of
  (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2,
  c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),  k += (W0, W1),
M0 = 0xD2511F53, M1 = 0xCD9E8D57, W0 = 0x9E3779B9, W1 = 0xBB67AE85.
Counter (index, stream, step lo, step hi), key = seed; uniforms (u+1)/2^32;
normals by Box-Muller: sqrt(-2 ln u0) (cos, sin)(2 pi u1) and
sqrt(-2 ln u2) cos(2 pi u3).  Streams: 0 ions, 2 body translation,
3 body rotation.

Hard spheres (section "Brownian dynamics", the potential-free hard-sphere
pair potential): every two particles closer than 2a -- ions, and beads of
different bodies -- interact through U(r) = gamma / (4 dt) (r - 2a)^2, so the
force on i from j is gamma / (2 dt) (2a - r) along (x_i - x_j) / r: under the
free-draining mobility 1/gamma one step separates an isolated overlapping
pair exactly to contact.  Beads of one rigid body never interact.

Rigid bodies (appendix "Force and torques derivation"): the body velocities
solve the saddle system of the bead mobility M^H and the rigid summation
tensor S3 (6 rows per body: the bead forces summed, and their moments
r x f): bead forces f with S3 f = (F, L) move the beads at
M^H f = S3^T (U, Omega) = U + Omega x r.  The printed block reads
[M^H, S3^T; S3, 0] [f_c; (U, Omega)] = [0; (F, L)]: with f_c the constraint
forces, that is the same system with (U, Omega) of the opposite sign, the
reading taken here.  With M^H = I / gamma it reduces per body to
U = F / (N gamma) (r measured from the centroid) and Omega = K^-1 L, the
free-draining update of ``step``.
"""
from __future__ import annotations

import math

import numpy as np

M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in counter)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def normals3(seed, step, index, stream):
    r = philox4x32_10((index, stream, step & MASK, (step >> 32) & MASK), (seed & MASK, (seed >> 32) & MASK))
    u = [(v + 1.0) * 2.0 ** -32 for v in r]
    a = math.sqrt(-2.0 * math.log(u[0]))
    b = math.sqrt(-2.0 * math.log(u[2]))
    return np.array([a * math.cos(2 * math.pi * u[1]), a * math.sin(2 * math.pi * u[1]),
                     b * math.cos(2 * math.pi * u[3])])


def quat_mul(p, q):
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rotvec_quat(th):
    ang = float(np.linalg.norm(th))
    if ang == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * th / ang])


def quat_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _min_image(d, box):
    return d - box * np.round(d / box)


def hard_sphere_forces(sys, a, gamma, dt):
    """(bead forces, ion forces) of the hard-sphere pair potential at the
    current positions, by brute force over all pairs (minimum image)."""
    box = np.asarray(sys.box, dtype=np.float64)
    pos = np.concatenate([sys.bead_pos, sys.ion_pos], 0)
    owner = np.concatenate([np.repeat(np.arange(sys.n_body), np.diff(sys.body_offsets)),
                            -1 - np.arange(sys.n_ion)])
    f = np.zeros_like(pos)
    for i in range(len(pos)):
        d = _min_image(pos[i] - pos, box)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        m = (r < 2 * a) & (owner != owner[i])
        if m.any():
            f[i] += ((gamma / (2 * dt)) * (2 * a - r[m]) / r[m]) @ d[m]
    return f[:sys.n_bead], f[sys.n_bead:]


def rigid_summation(rel, body_offsets):
    """The rigid summation tensor (6 n_body x 3 n_bead): rows 6i..6i+2 sum
    body i's bead forces, rows 6i+3..6i+5 their moments r x f."""
    off = np.asarray(body_offsets, dtype=np.int64)
    nb = len(off) - 1
    S = np.zeros((6 * nb, 3 * off[-1]))
    for i in range(nb):
        for j in range(off[i], off[i + 1]):
            S[6 * i:6 * i + 3, 3 * j:3 * j + 3] = np.eye(3)
            x, y, z = rel[j]
            S[6 * i + 3:6 * i + 6, 3 * j:3 * j + 3] = np.array([[0, -z, y], [z, 0, -x], [-y, x, 0]])
    return S


def rigid_velocities(rel, body_offsets, body_force, body_torque, mobility):
    """(U, Omega) per body from the dense saddle system of the bead mobility
    (3 n_bead square) and the rigid summation tensor."""
    S = rigid_summation(rel, body_offsets)
    nb = S.shape[0] // 6
    A = np.block([[mobility, -S.T], [S, np.zeros((6 * nb, 6 * nb))]])
    FL = np.concatenate([np.concatenate([body_force[i], body_torque[i]]) for i in range(nb)])
    x = np.linalg.solve(A, np.concatenate([np.zeros(S.shape[1]), FL]))
    V = x[S.shape[1]:].reshape(nb, 6)
    return V[:, :3], V[:, 3:]


def step(sys, body_force, body_torque, ion_force, dt, kT, gamma, seed, step_no, hs_radius=0.0):
    """Return new (bead_pos, body_center, body_quat, ion_pos).  With
    hs_radius > 0 the hard-sphere forces at the current positions are added
    to the given forces (their bead parts summed into each body's force and
    its torque about the centre)."""
    if hs_radius > 0:
        fb, fi = hard_sphere_forces(sys, hs_radius, gamma, dt)
        ion_force = np.asarray(ion_force, dtype=np.float64) + fi
        body_force = np.array(body_force, dtype=np.float64)
        body_torque = np.array(body_torque, dtype=np.float64)
        for b in range(sys.n_body):
            o0, o1 = sys.body_offsets[b], sys.body_offsets[b + 1]
            r = sys.bead_pos[o0:o1] - sys.body_center[b]
            body_force[b] += fb[o0:o1].sum(0)
            body_torque[b] += np.cross(r, fb[o0:o1]).sum(0)
    ion = sys.ion_pos.copy()
    s = math.sqrt(2 * kT * dt / gamma)
    for i in range(sys.n_ion):
        ion[i] += ion_force[i] * dt / gamma + s * normals3(seed, step_no, i, 0)
    X = sys.body_center.copy()
    Q = sys.body_quat.copy()
    pos = sys.bead_pos.copy()
    off = sys.body_offsets
    for b in range(sys.n_body):
        r = sys.bead_pos[off[b]:off[b + 1]] - sys.body_center[b]
        N = len(r)
        X[b] = X[b] + body_force[b] * dt / (N * gamma) + math.sqrt(2 * kT * dt / (N * gamma)) * normals3(
            seed, step_no, b, 2)
        K = gamma * (np.sum(r * r) * np.eye(3) - r.T @ r)
        Ki = np.linalg.inv(K)
        C = np.linalg.cholesky(0.5 * (Ki + Ki.T))
        th = Ki @ body_torque[b] * dt + math.sqrt(2 * kT * dt) * C @ normals3(seed, step_no, b, 3)
        dq = rotvec_quat(th)
        Q[b] = quat_mul(dq, Q[b])
        Q[b] /= np.linalg.norm(Q[b])
        pos[off[b]:off[b + 1]] = X[b] + r @ quat_matrix(dq).T
    return pos, X, Q, ion
