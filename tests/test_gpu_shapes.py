"""Rigid-shape handling of the Krylov operator against the dense discrete
operator of the oracle (mode B).

Bodies of one shape share a dense intra-body real-space block; bodies of
different shapes, widths or sizes get blocks of their own; a body wider than
half the box keeps its intra-body pairs in the sparse list.  In every case the
saddle operator must equal the dense discrete saddle matrix times x, in double
to rounding and in float to the float bound.
"""
import numpy as np
import pytest

from oracle import saddle, se
from paper_2401_04865_amd import inputs

pytestmark = pytest.mark.gpu


def _system(shapes, sigmas, L, seed, n_ion=12, mesh=(32, 32, 32)):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(shapes)
    centers = inputs.rsa_centers(rng, [L] * 3, n, 2.3)
    quats = inputs.random_quaternions(rng, n)
    ip, iq, isg = inputs.place_ions(rng, [L] * 3, n_ion // 2, n_ion - n_ion // 2, centers, 1.2, sigma=0.1)
    s = inputs.assemble(L, shapes, centers, quats, np.linspace(-0.3, 0.4, n), np.arange(n) % 2, sigmas[0],
                        ip, iq, isg, E0=inputs.random_unit_vector(rng), mesh=mesh, name=f"shapes{seed}")
    # per-body widths
    sig = np.concatenate([np.full(len(sh), sg) for sh, sg in zip(shapes, sigmas)])
    s.bead_sigma = sig
    return s


def _check_operator(gpu_lib, s, P=8, split_tol=1e-10):
    import torch
    B = gpu_lib
    A = None
    for prec, tol in ((B.PE_FP64, 1e-11), (B.PE_MIXED, 3e-6)):
        p = B.make_params(s.box, s.mesh, P=P, split_tol=split_tol, precision=prec)
        ctx = B.Context(p).load(s)
        d = ctx.pe_get_derived()
        if A is None:
            M = se.matrix(s.bead_pos, s.bead_sigma, s.box, s.mesh, P, d["xi"], d["eta"], d["r_cut"])
            A = saddle.saddle_matrix(M, s.body_offsets)
        x = np.random.default_rng(3).standard_normal(A.shape[0])
        y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
        ctx.pe_apply_saddle(torch.as_tensor(x, device="cuda"), y, prec)
        ref = A @ x
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        print("precision", prec, "rel err", err, "r_cut", d["r_cut"])
        assert err <= tol
        ctx.close()
    return d


def test_mixed_shapes_share_and_separate_blocks(gpu_lib):
    """Two icospheres of one shape (turned differently), one of the same
    geometry but other widths, a short rod and a small cube: four shapes."""
    sph = inputs.icosphere(1, 0.7)
    rod = inputs.rod(length=1.4, diameter=0.6, spacing=0.25)
    cube = inputs.cube(edge=1.0, n=3)
    s = _system([sph, sph, sph, rod, cube], [0.15, 0.15, 0.12, 0.15, 0.15], L=8.0, seed=5, mesh=(40, 40, 40))
    d = _check_operator(gpu_lib, s)
    # every intra-body distance is inside r_c here, so the dense blocks and the
    # truncated oracle describe the same pairs
    for b in range(s.n_body):
        seg = s.bead_pos[s.body_offsets[b]:s.body_offsets[b + 1]]
        span = np.sqrt(((seg[:, None, :] - seg[None, :, :]) ** 2).sum(-1)).max()
        assert span < d["r_cut"]
    # the intra-body pairs are held by the dense blocks, not the sparse list
    intra = sum(int(n) ** 2 for n in np.diff(s.body_offsets))
    assert d["nnz"] < intra


def test_body_wider_than_half_box_uses_sparse_pairs(gpu_lib):
    """A rod longer than a quarter box per side keeps its intra-body pairs in
    the sparse list (truncated at r_c like the oracle)."""
    rod = inputs.rod(length=3.8, diameter=0.6, spacing=0.3)
    sph = inputs.icosphere(1, 0.7)
    s = _system([rod, sph], [0.15, 0.15], L=7.0, seed=9, mesh=(32, 32, 32))
    d = _check_operator(gpu_lib, s)
    # the configuration really exercises the sparse path: the rod is longer
    # than r_c, which only the truncated sparse list reproduces
    seg = s.bead_pos[s.body_offsets[0]:s.body_offsets[1]]
    span = np.sqrt(((seg[:, None, :] - seg[None, :, :]) ** 2).sum(-1)).max()
    assert span > d["r_cut"]
    n_rod = int(s.body_offsets[1])
    assert d["nnz"] >= n_rod  # at least the rod's own pairs (its self pairs included)


def test_pair_structure_kept_across_small_moves(gpu_lib):
    """The bead-bead pair structure is built with a skin beyond r_c and kept
    while no bead has moved more than half the skin; its values are
    recomputed from the current positions every time.  After a small rigid
    move (structure kept) and after a large one (structure rebuilt) the
    saddle operator equals the dense discrete saddle matrix at the new
    positions."""
    import copy
    import torch
    B = gpu_lib
    sph = inputs.icosphere(1, 0.7)
    rod = inputs.rod(length=1.4, diameter=0.6, spacing=0.25)
    s0 = _system([sph, sph, rod], [0.15, 0.12, 0.15], L=8.0, seed=31, mesh=(40, 40, 40))
    rng = np.random.default_rng(41)
    for prec, tol in ((B.PE_FP64, 1e-11), (B.PE_MIXED, 3e-6)):
        p = B.make_params(s0.box, s0.mesh, P=8, split_tol=1e-8, precision=prec)
        ctx = B.Context(p)
        s = copy.deepcopy(s0)
        for step, shift in enumerate((0.0, 0.004, 0.6)):
            # rigid translation of every body by its own random direction
            for b in range(s.n_body):
                o0, o1 = s.body_offsets[b], s.body_offsets[b + 1]
                dvec = rng.standard_normal(3)
                dvec *= shift / np.linalg.norm(dvec)
                s.bead_pos[o0:o1] += dvec
                s.body_center[b] += dvec
            ctx.load(s)
            d = ctx.pe_get_derived()
            assert d["ncell"] >= 3  # three or more cells per axis: the skin is in use
            M = se.matrix(s.bead_pos, s.bead_sigma, s.box, s.mesh, 8, d["xi"], d["eta"], d["r_cut"])
            A = saddle.saddle_matrix(M, s.body_offsets)
            x = np.random.default_rng(step).standard_normal(A.shape[0])
            y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
            ctx.pe_apply_saddle(torch.as_tensor(x, device="cuda"), y, prec)
            ref = A @ x
            err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
            print(prec, step, err, d["nnz"])
            assert err <= tol
        ctx.close()


def test_saddle_operator_full_size_sampled_sources(gpu_lib):
    """The Krylov operator at full size (512 bodies of 642 beads, the
    per-shape near-field product over all of them on the matrix cores, split
    over K): with bead charges on 40 beads of four bodies and no potential
    offsets, the bead rows at 40 other beads of the same bodies equal minus
    the oracle's potential from those sources, and the body rows equal the
    bodies' charge sums.  A body's dense block keeps all of its own pairs
    (the sphere is wider than r_c), so the reference adds, per body, the
    oracle's real-space sum over the same pairs beyond r_c."""
    import torch
    B = gpu_lib
    s = inputs.config(5)
    pos, sig, _ = saddle.all_particles(s, np.zeros(s.n_bead))
    rng = np.random.default_rng(53)
    bodies = rng.choice(s.n_body, 4, replace=False)
    src, tgt = [], []
    for b in bodies:
        beads = np.arange(s.body_offsets[b], s.body_offsets[b + 1])
        pick = rng.choice(beads, 20, replace=False)
        src += list(pick[:10])
        tgt += list(pick[10:])
    src, tgt = np.array(src), np.array(tgt)
    q = rng.standard_normal(len(src))
    n = s.n_bead + s.n_body
    x = np.zeros(n)
    x[src] = q
    ref = None
    for prec, tol in ((B.PE_FP64, 1e-10), (B.PE_MIXED, 3e-6)):
        p = B.make_params(s.box, s.mesh, P=8, split_tol=1e-6, precision=prec)
        ctx = B.Context(p).load(s)
        d = ctx.pe_get_derived()
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        ctx.pe_apply_saddle(torch.as_tensor(x, device="cuda"), y, prec)
        y = y.cpu().numpy()
        ctx.close()
        if ref is None:
            ref, _ = se.apply(pos[tgt], sig[tgt], pos[src], sig[src], q, s.box, s.mesh, 8, d["xi"], d["eta"],
                              d["r_cut"], want_field=False, same=False)
            for k in range(len(bodies)):
                t, sr = slice(10 * k, 10 * k + 10), slice(10 * k, 10 * k + 10)
                far, _ = se.real_potential(pos[tgt[t]], sig[tgt[t]], pos[src[sr]], sig[src[sr]], q[sr], s.box,
                                           d["xi"], 0.49 * min(s.box))
                near, _ = se.real_potential(pos[tgt[t]], sig[tgt[t]], pos[src[sr]], sig[src[sr]], q[sr], s.box,
                                            d["xi"], d["r_cut"])
                ref[t] += far - near
        err = np.abs(-y[tgt] - ref).max() / np.abs(ref).max()
        print(prec, err)
        assert err <= tol
        sums = np.array([x[s.body_offsets[b]:s.body_offsets[b + 1]].sum() for b in range(s.n_body)])
        np.testing.assert_allclose(y[s.n_bead:], sums, rtol=0, atol=1e-12)
