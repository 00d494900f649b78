"""Seeded synthetic inputs: body geometry, ion clouds and whole systems.

This module builds *inputs only*.  It holds none of the electrostatics (no
potentials, no Ewald sums, no solves), so both the HIP path and the CPU
oracle may consume what it produces without sharing any of the method's
arithmetic.

Geometry follows the composite-bead model of the paper (section "Composite
Bead Model"): a body is a rigid set of bead centres on its surface; spheres
are icospheres (12 icosahedron vertices, edges bisected and the new points
projected back onto the sphere, repeated ``level`` times).  Ions are bodies
of a single bead (section "Induced Surface Charge Distribution").

All randomness is NumPy ``PCG64`` seeded by the caller, so every system is
reproducible bit for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# Body shapes (body frame, centroid at the origin)
# --------------------------------------------------------------------------


def icosphere(level: int, radius: float = 1.0) -> np.ndarray:
    """Bead centres of a level-``level`` icosphere of the given radius.

    Level 0 is the icosahedron (12 beads); each level bisects every edge and
    projects the midpoints radially onto the sphere: 12, 42, 162, 642, 2562.
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
         (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
         (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        new_faces = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    return radius * np.asarray(verts)


def rod(length: float = 4.0, diameter: float = 1.0, spacing: float = 0.12) -> np.ndarray:
    """Closed cylinder along z: a grid of beads on the lateral surface plus
    concentric rings on the two flat caps (about 1000 beads for 4 x 1)."""
    r = diameter / 2.0
    n_around = max(3, int(round(2 * math.pi * r / spacing)))
    n_along = max(2, int(round(length / spacing)) + 1)
    pts = []
    zs = np.linspace(-length / 2, length / 2, n_along)
    for iz, z in enumerate(zs):
        off = 0.5 * (iz % 2)  # staggered rows
        for k in range(n_around):
            t = 2 * math.pi * (k + off) / n_around
            pts.append((r * math.cos(t), r * math.sin(t), z))
    # caps: rings of radius r_k = k*spacing (k>=1, strictly inside), plus the centre
    n_rings = int(math.floor(r / spacing - 0.5))
    for zc in (-length / 2, length / 2):
        pts.append((0.0, 0.0, zc))
        for k in range(1, n_rings + 1):
            rk = k * spacing
            nk = max(3, int(round(2 * math.pi * rk / spacing)))
            for j in range(nk):
                t = 2 * math.pi * j / nk
                pts.append((rk * math.cos(t), rk * math.sin(t), zc))
    p = np.asarray(pts, dtype=np.float64)
    return p - p.mean(axis=0)


def cube(edge: float = 2.0, n: int = 13) -> np.ndarray:
    """n x n beads at the face-cell centres of each of the six faces."""
    h = edge / n
    c = (np.arange(n) + 0.5) * h - edge / 2
    u, v = np.meshgrid(c, c, indexing="ij")
    u, v = u.ravel(), v.ravel()
    w = np.full_like(u, edge / 2)
    faces = [np.stack([w, u, v], 1), np.stack([-w, u, v], 1),
             np.stack([u, w, v], 1), np.stack([u, -w, v], 1),
             np.stack([u, v, w], 1), np.stack([u, v, -w], 1)]
    p = np.concatenate(faces, 0)
    return p - p.mean(axis=0)


def min_bead_spacing(p: np.ndarray) -> float:
    """Smallest centre-to-centre distance among the beads of one body."""
    d = np.linalg.norm(p[:, None, :] - p[None, :, :], axis=-1)
    d[np.diag_indices_from(d)] = np.inf
    return float(d.min())


# --------------------------------------------------------------------------
# Rotations
# --------------------------------------------------------------------------


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed unit quaternions (w, x, y, z)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    return q


def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices (n,3,3) for unit quaternions (n,4) in (w,x,y,z) order."""
    q = np.atleast_2d(q)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_unit_vector(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# Systems
# --------------------------------------------------------------------------


@dataclass
class System:
    """A periodic system of rigid conducting bodies and fixed-charge ions.

    Beads are stored body-major; ``body_offsets[i]:body_offsets[i+1]`` are the
    beads of body i.  Positions are unwrapped lab-frame coordinates: a bead
    sits at ``body_center[i] + R_i @ body_frame_bead``.
    """
    box: np.ndarray                  # (3,) box lengths
    body_offsets: np.ndarray         # (n_body+1,) int64
    bead_pos: np.ndarray             # (n_bead,3)
    bead_sigma: np.ndarray           # (n_bead,)
    bead_ref: np.ndarray             # (n_bead,3) body-frame bead coordinates
    body_center: np.ndarray          # (n_body,3)
    body_quat: np.ndarray            # (n_body,4) (w,x,y,z)
    body_charge: np.ndarray          # (n_body,)
    body_type: np.ndarray            # (n_body,) int32 shape id
    ion_pos: np.ndarray              # (n_ion,3)
    ion_charge: np.ndarray           # (n_ion,)
    ion_sigma: np.ndarray            # (n_ion,)
    E0: np.ndarray                   # (3,)
    mesh: tuple = (32, 32, 32)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_body(self) -> int:
        return len(self.body_offsets) - 1

    @property
    def n_bead(self) -> int:
        return int(self.body_offsets[-1])

    @property
    def n_ion(self) -> int:
        return len(self.ion_charge)


def assemble(box, shapes, centers, quats, charges, types, sigma_bead,
             ion_pos=None, ion_charge=None, ion_sigma=None, E0=(0, 0, 1),
             mesh=(32, 32, 32), name="") -> System:
    """Place body-frame shapes at centres with rotations and stack them."""
    box = np.asarray(box, dtype=np.float64)
    if box.ndim == 0:
        box = np.full(3, float(box))
    Rs = quat_to_matrix(np.asarray(quats, dtype=np.float64))
    pos, ref, offs = [], [], [0]
    for s, c, R in zip(shapes, centers, Rs):
        ref.append(s)
        pos.append(np.asarray(c) + s @ R.T)
        offs.append(offs[-1] + len(s))
    n = offs[-1]
    if ion_pos is None:
        ion_pos = np.zeros((0, 3))
        ion_charge = np.zeros(0)
        ion_sigma = np.zeros(0)
    return System(
        box=box,
        body_offsets=np.asarray(offs, dtype=np.int64),
        bead_pos=np.concatenate(pos, 0) if pos else np.zeros((0, 3)),
        bead_sigma=np.full(n, float(sigma_bead)),
        bead_ref=np.concatenate(ref, 0) if ref else np.zeros((0, 3)),
        body_center=np.asarray(centers, dtype=np.float64).reshape(-1, 3),
        body_quat=np.asarray(quats, dtype=np.float64).reshape(-1, 4),
        body_charge=np.asarray(charges, dtype=np.float64),
        body_type=np.asarray(types, dtype=np.int32),
        ion_pos=np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3),
        ion_charge=np.asarray(ion_charge, dtype=np.float64),
        ion_sigma=np.asarray(ion_sigma, dtype=np.float64),
        E0=np.asarray(E0, dtype=np.float64),
        mesh=tuple(int(m) for m in mesh),
        name=name,
    )


def _min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.round(d / box)


def place_ions(rng, box, n_pos, n_neg, centers, exclusion, sigma=0.1,
               bead_pos=None, bead_exclusion=0.0, batch=200_000):
    """Uniform ions in [0,L)^3 with charges +1 (n_pos) and -1 (n_neg),
    rejected within ``exclusion`` (minimum image) of any body centre and, if
    ``bead_pos`` is given, within ``bead_exclusion`` of any bead."""
    from scipy.spatial import cKDTree

    box = np.asarray(box, dtype=np.float64)
    need = n_pos + n_neg
    ctree = cKDTree(np.mod(centers, box), boxsize=box) if len(centers) else None
    btree = (cKDTree(np.mod(bead_pos, box), boxsize=box)
             if bead_pos is not None and bead_exclusion > 0 else None)
    out = []
    have = 0
    while have < need:
        cand = rng.random((batch, 3)) * box
        ok = np.ones(batch, dtype=bool)
        # only whether a neighbour lies within the exclusion matters, so the
        # searches stop there (a candidate with none gets d = inf)
        if ctree is not None:
            d, _ = ctree.query(cand, k=1, distance_upper_bound=exclusion)
            ok &= d >= exclusion
        if btree is not None:
            d, _ = btree.query(cand, k=1, distance_upper_bound=bead_exclusion)
            ok &= d >= bead_exclusion
        cand = cand[ok][: need - have]
        out.append(cand)
        have += len(cand)
    pos = np.concatenate(out, 0) if out else np.zeros((0, 3))
    q = np.concatenate([np.ones(n_pos), -np.ones(n_neg)])
    return pos, q, np.full(need, float(sigma))


def rsa_centers(rng, box, n, min_sep, max_tries=2_000_000):
    """Random sequential addition of n centres with minimum-image separation."""
    box = np.asarray(box, dtype=np.float64)
    pts = np.zeros((0, 3))
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA failed to place all centres")
        c = rng.random(3) * box
        if len(pts):
            d = np.linalg.norm(_min_image(pts - c, box), axis=1)
            if d.min() < min_sep:
                continue
        pts = np.vstack([pts, c])
    return pts


def _rsa_mixed(rng, box, radii, max_tries=5_000_000):
    """RSA for bodies with individual bounding radii."""
    box = np.asarray(box, dtype=np.float64)
    pts = np.zeros((0, 3))
    rad = []
    tries = 0
    for r in radii:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("RSA failed")
            c = rng.random(3) * box
            if len(pts):
                d = np.linalg.norm(_min_image(pts - c, box), axis=1)
                if np.any(d < np.asarray(rad) + r):
                    continue
            pts = np.vstack([pts, c])
            rad.append(r)
            break
    return pts


SEED_BASE = 20240109


def config(k: int, seed: int | None = None, **over) -> System:
    """The five synthetic workloads (k = 1..5) and their stated readings.

    1: one level-2 icosphere (R=1, sigma 0.2) at the centre of L=20, E0 = z.
    2: two level-3 icospheres (sigma 0.05) 2.5 apart on z, 1000+1000 ions
       (sigma 0.1), L=30, mesh 64.
    3: 4^3 simple-cubic lattice of level-3 spheres (phi = 0.2), 20k+20k ions,
       mesh 128, E0 a seeded random unit vector.
    4: 128 rods (4 x 1) + 128 cubes (edge 2), 50k+50k ions, L=32, mesh 192.
    5: 512 level-3 spheres with Q=+20, 10240 counterions + 494880 salt pairs,
       phi = 0.1, mesh 256, E0 = 0.5 z.
    """
    seed = SEED_BASE + k if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    if k == 1:
        L = over.get("L", 20.0)
        s = icosphere(2, 1.0)
        c = np.full((1, 3), L / 2)
        return assemble(L, [s], c, [[1, 0, 0, 0]], [0.0], [0],
                        over.get("sigma", 0.2), E0=(0, 0, 1),
                        mesh=over.get("mesh", (32, 32, 32)), name="cfg1")
    if k == 2:
        L = over.get("L", 30.0)
        sep = over.get("sep", 2.5)
        s = icosphere(3, 1.0)
        c = np.array([[L / 2, L / 2, L / 2 - sep / 2], [L / 2, L / 2, L / 2 + sep / 2]])
        n_ion = over.get("n_ion", 2000)
        ip, iq, isg = place_ions(rng, [L] * 3, n_ion // 2, n_ion // 2, c, 1.2)
        return assemble(L, [s, s], c, [[1, 0, 0, 0]] * 2, [0.0, 0.0], [0, 0],
                        over.get("sigma", 0.05), ip, iq, isg, E0=(0, 0, 1),
                        mesh=over.get("mesh", (64, 64, 64)), name="cfg2")
    if k == 3:
        nside = over.get("nside", 4)
        d = (4 * math.pi / (3 * 0.2)) ** (1 / 3)
        L = nside * d
        s = icosphere(over.get("level", 3), 1.0)
        g = (np.arange(nside) + 0.5) * d
        c = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        n_ion = over.get("n_ion", 40000)
        ip, iq, isg = place_ions(rng, [L] * 3, n_ion // 2, n_ion // 2, c, 1.2)
        E0 = random_unit_vector(rng)
        nb = len(c)
        return assemble(L, [s] * nb, c, [[1, 0, 0, 0]] * nb, np.zeros(nb), np.zeros(nb),
                        over.get("sigma", 0.05), ip, iq, isg, E0=E0,
                        mesh=over.get("mesh", (128, 128, 128)), name="cfg3")
    if k == 4:
        L = over.get("L", 32.0)
        n_rod = over.get("n_rod", 128)
        n_cube = over.get("n_cube", 128)
        srod, scube = rod(), cube()
        radii = [2.06] * n_rod + [1.73] * n_cube
        order = rng.permutation(len(radii))
        radii = [radii[i] for i in order]
        c = _rsa_mixed(rng, [L] * 3, radii)
        types = np.array([0 if r > 2.0 else 1 for r in radii], dtype=np.int32)
        shapes = [srod if t == 0 else scube for t in types]
        quats = random_quaternions(rng, len(radii))
        sysb = assemble(L, shapes, c, quats, np.zeros(len(radii)), types, over.get("sigma", 0.05),
                        mesh=over.get("mesh", (192, 192, 192)))
        n_ion = over.get("n_ion", 100000)
        ip, iq, isg = place_ions(rng, [L] * 3, n_ion // 2, n_ion // 2, np.zeros((0, 3)), 0.0,
                                 bead_pos=sysb.bead_pos, bead_exclusion=0.2,
                                 batch=over.get("ion_batch", 200_000))
        E0 = random_unit_vector(rng)
        return assemble(L, shapes, c, quats, np.zeros(len(radii)), types, over.get("sigma", 0.05),
                        ip, iq, isg, E0=E0, mesh=over.get("mesh", (192, 192, 192)), name="cfg4")
    if k == 5:
        n_sph = over.get("n_body", 512)
        phi = over.get("phi", 0.1)
        L = (n_sph * 4 * math.pi / 3 / phi) ** (1 / 3)
        s = icosphere(3, 1.0)
        c = rsa_centers(rng, [L] * 3, n_sph, 2.2)
        Q = over.get("Q", 20.0)
        n_counter = int(round(n_sph * Q))
        n_total = over.get("n_ion", 1_000_000)
        n_salt = (n_total - n_counter) // 2
        ip, iq, isg = place_ions(rng, [L] * 3, n_salt, n_salt + n_counter, c, 1.2)
        return assemble(L, [s] * n_sph, c, [[1, 0, 0, 0]] * n_sph, np.full(n_sph, Q),
                        np.zeros(n_sph), over.get("sigma", 0.05), ip, iq, isg,
                        E0=(0, 0, 0.5), mesh=over.get("mesh", (256, 256, 256)), name="cfg5")
    raise ValueError(f"unknown config {k}")


def training_system(seed: int, n_body: int = 32, n_ion: int = 12500, L: float = 16.0,
                    mesh=(96, 96, 96)) -> System:
    """Reduced-scale system of the cfg4 kind (rods and cubes at the same
    density): the source of training solves for the learned initial guess."""
    return config(4, seed=seed, L=L, n_rod=n_body // 2, n_cube=n_body - n_body // 2,
                  n_ion=n_ion, mesh=mesh, ion_batch=2 * n_ion)


def training_spheres(seed: int, n_body: int = 64, mesh=(128, 128, 128)) -> System:
    """Reduced-scale system of the 512-sphere kind (charged level-3 spheres,
    volume fraction 0.1, the same ion density and grid spacing): training
    solves for the learned warm start of the Brownian-dynamics workload."""
    n_ion = int(round(1_000_000 * n_body / 512))
    return config(5, seed=seed, n_body=n_body, n_ion=n_ion, mesh=mesh)


def small_random_system(seed: int, n_body: int = 2, level: int = 1, n_ion: int = 20,
                        L: float = 6.0, sigma: float = 0.15, ion_sigma: float = 0.1,
                        charges=None, mesh=(16, 16, 16), E0=None) -> System:
    """A tiny system for brute-force checks: a few small icospheres with random
    orientation, a handful of ions, a random field."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = icosphere(level, 0.8)
    c = rsa_centers(rng, [L] * 3, n_body, 2.0)
    quats = random_quaternions(rng, n_body)
    ip, iq, isg = place_ions(rng, [L] * 3, n_ion // 2, n_ion - n_ion // 2, c, 1.0, sigma=ion_sigma)
    if charges is None:
        charges = np.zeros(n_body)
    if E0 is None:
        E0 = random_unit_vector(rng)
    return assemble(L, [s] * n_body, c, quats, charges, np.zeros(n_body), sigma,
                    ip, iq, isg, E0=E0, mesh=mesh, name=f"small{seed}")
