"""Seeded input generators: mesh validity, conformity, Dirichlet masks,
indenter seating at initial contact, draw ranges and reproducibility."""
import math

import numpy as np
import pytest

from paper_2103_16747_amd import workload as W


def face_counts(tets):
    faces = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]]),
                    axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    return counts


def test_cube_block_sizes_and_orientation(oracle_lib):
    m = W.cube_block_mesh()
    assert (m.n, m.m, int(m.fixed.sum())) == (729, 3072, 81)
    rc, B, V = oracle_lib.precompute(m.X, m.tets)
    assert rc == 0 and np.all(V > 0)
    assert set(face_counts(m.tets)) <= {1, 2}


@pytest.mark.parametrize("target", [5000, 20000, 50000, 120000])
def test_fingertip_meshes(oracle_lib, target):
    m = W.fingertip_mesh(target)
    assert abs(m.m - target) <= 0.05 * target
    rc, B, V = oracle_lib.precompute(m.X, m.tets)
    assert rc == 0 and np.all(V > 0)
    counts = face_counts(m.tets)
    assert set(counts) <= {1, 2}                     # conforming: no face in 3+ tets
    assert np.all(m.fixed[m.X[:, 2] == 0.0] == 1)      # clamped base
    rho = np.hypot(m.X[:, 0], m.X[:, 1])
    inner = (m.X[:, 2] < W.FT_L_CYL) & (rho < W.FT_R_IN)
    assert np.all(m.fixed[inner] == 1)                 # bonded to the core
    outer = rho > W.FT_R_OUT - 1e-9
    assert np.all(m.fixed[outer & (m.X[:, 2] > 0.0)] == 0)


def test_random_indentation_ranges_and_reproducibility():
    for seed in range(2000, 2040):
        a = W.random_indentation(seed)
        b = W.random_indentation(seed)
        assert a.kind == b.kind and np.array_equal(a.shape, b.shape) and np.array_equal(a.c0, b.c0)
        assert 0.0 <= a.depth <= 3e-3 and a.steps == 100
        assert abs(np.linalg.det(a.R) - 1) < 1e-12 and np.allclose(a.R.T @ a.R, np.eye(3), atol=1e-12)
        assert np.allclose(a.R[:, 2], a.direction, atol=1e-12)
        p = a.contact_point
        assert p[2] >= 5e-3 - 1e-12
        # outward design-surface normal at p, then the tilt bound
        if p[2] <= W.FT_L_CYL:
            n = np.array([p[0], p[1], 0.0])
            assert abs(np.linalg.norm(n) - W.FT_R_OUT) < 1e-12
        else:
            n = np.array([p[0] / W.FT_R_OUT ** 2, p[1] / W.FT_R_OUT ** 2, (p[2] - W.FT_L_CYL) / W.FT_C_OUT ** 2])
        n /= np.linalg.norm(n)
        assert math.degrees(math.acos(min(1.0, -a.direction @ n))) <= 30.0 + 1e-9


@pytest.mark.parametrize("seed", range(3000, 3012))
def test_seating_touches_without_penetration(oracle_lib, seed):
    mesh = W.fingertip_mesh(5000)
    ind = W.seat_on_mesh(W.random_indentation(seed), mesh)
    I = oracle_lib.make_indenter(ind.kind, ind.shape, ind.R, ind.c0)
    free = np.nonzero(mesh.fixed == 0)[0]
    phi = np.array([oracle_lib.sdf(I, mesh.X[i])[0] for i in free])
    assert phi.min() >= -1e-12 and phi.min() <= 1e-12


def test_xoshiro_stream_properties():
    r = W.Xoshiro256ss(12345)
    xs = np.array([r.uniform() for _ in range(20000)])
    assert xs.min() >= 0.0 and xs.max() < 1.0
    assert abs(xs.mean() - 0.5) < 0.01 and abs(xs.var() - 1 / 12) < 0.005
    assert W.Xoshiro256ss(1).next_u64() != W.Xoshiro256ss(2).next_u64()


def test_poisson_arrivals():
    t = W.poisson_arrivals(7, 50.0, 4000)
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1 / 50.0) < 0.002
