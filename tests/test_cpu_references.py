"""Pins of the CPU references used by the GPU tests of the learned guess and
of the Brownian-dynamics step."""
import json
import os

import numpy as np

from oracle import bd, mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        c = [int(x, 16) for x in v["counter"]]
        k = [int(x, 16) for x in v["key"]]
        assert list(bd.philox4x32_10(c, k)) == [int(x, 16) for x in v["out"]]


def test_box_muller_normals_statistics():
    g = np.array([bd.normals3(7, 3, i, 0) for i in range(4000)]).ravel()
    assert abs(g.mean()) < 0.05 and abs(g.std() - 1.0) < 0.05


def _rows(n, seed=0):
    rng = np.random.default_rng(seed)
    rows = np.zeros((n, 11))
    rows[:, :3] = rng.standard_normal((n, 3))
    rows[:, 3:6] = rng.standard_normal((n, 3))
    t = rng.integers(0, 2, n)
    rows[:, 6] = t == 0
    rows[:, 7] = t == 1
    rows[:, 8] = rng.standard_normal(n) * 0.01
    rows[:, 9] = rng.standard_normal(n) * 0.1
    return rows


def test_mlp_reference_gradient_by_central_differences():
    rng = np.random.default_rng(1)
    P = rng.standard_normal(mlp.NPAR) * 0.2
    rows = _rows(40)
    L, g = mlp.loss_grad(P, rows)
    h = 1e-6
    idx = rng.choice(mlp.NPAR, 60, replace=False)
    idx = np.concatenate([idx, [mlp.ob3 - 1, mlp.NPAR - 1, mlp.oW2 + 5, mlp.ob1]])
    for i in idx:
        e = np.zeros(mlp.NPAR)
        e[i] = h
        fd = (mlp.loss_grad(P + e, rows)[0] - mlp.loss_grad(P - e, rows)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g).max()), i


def test_rigid_body_step_keeps_shape_and_charge_free_translation():
    """A zero-temperature step moves a body rigidly: its bead distances are
    unchanged and the centre moves by F dt / (N gamma)."""
    from paper_2401_04865_amd import inputs
    s = inputs.small_random_system(3, n_body=1, level=1, n_ion=2, L=8.0)
    F = np.array([[0.3, -0.2, 0.5]])
    L = np.array([[0.01, 0.02, -0.03]])
    pos, X, Q, ion = bd.step(s, F, L, np.zeros((2, 3)), 0.01, 0.0, 1.0, 5, 0)
    d0 = np.linalg.norm(s.bead_pos[:, None] - s.bead_pos[None], axis=-1)
    d1 = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    np.testing.assert_allclose(d1, d0, atol=1e-12)
    np.testing.assert_allclose(X[0] - s.body_center[0], F[0] * 0.01 / 42, atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(Q[0]), 1.0, atol=1e-14)
