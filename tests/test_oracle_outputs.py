"""Pins of the oracle's data-generation outputs: per-tet Cauchy and von Mises
stress and the displacement-norm statistics (paper Sec. IV reports the
maximum and mean nodal displacement norm per indentation).

Checks against closed forms of the compressible Neo-Hookean law
(sigma = [mu (B - I) + lam ln J I] / J), rotation and objectivity, the
small-strain shear limit, a homogeneous deformation of a whole mesh, and
brute-force statistics.
"""
import numpy as np

from paper_2103_16747_amd import workload as W
from test_oracle_pins import rand_rotation

E0, NU0 = 0.3e6, 0.45


def closed_form(F, mu, lam):
    J = np.linalg.det(F)
    B = F @ F.T
    S = (mu * (B - np.eye(3)) + lam * np.log(J) * np.eye(3)) / J
    return S


def six(S):
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]])


def von_mises(S):
    dev = S - np.trace(S) / 3.0 * np.eye(3)
    return float(np.sqrt(1.5 * np.sum(dev * dev)))


def full(s):
    return np.array([[s[0], s[3], s[4]], [s[3], s[1], s[5]], [s[4], s[5], s[2]]])


def test_cauchy_matches_closed_form(oracle_lib):
    mu, lam = oracle_lib.lame(E0, NU0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0.2:
            continue
        S = closed_form(F, mu, lam)
        s, vm = oracle_lib.cauchy(F, mu, lam)
        assert np.abs(s - six(S)).max() <= 1e-10 * np.abs(S).max()
        assert abs(vm - von_mises(S)) <= 1e-10 * np.abs(S).max()


def test_rigid_rotation_is_stress_free(oracle_lib):
    mu, lam = oracle_lib.lame(E0, NU0)
    Q = rand_rotation(np.random.default_rng(5))
    s, vm = oracle_lib.cauchy(Q, mu, lam)
    assert np.abs(s).max() <= 1e-9 * mu and vm <= 1e-9 * mu


def test_stress_is_objective(oracle_lib):
    mu, lam = oracle_lib.lame(E0, NU0)
    rng = np.random.default_rng(11)
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    Q = rand_rotation(rng)
    s1, vm1 = oracle_lib.cauchy(F, mu, lam)
    s2, vm2 = oracle_lib.cauchy(Q @ F, mu, lam)
    assert np.abs(full(s2) - Q @ full(s1) @ Q.T).max() <= 1e-10 * np.abs(s1).max()
    assert abs(vm1 - vm2) <= 1e-10 * vm1


def test_hydrostatic_state_has_no_von_mises_stress(oracle_lib):
    mu, lam = oracle_lib.lame(E0, NU0)
    s, vm = oracle_lib.cauchy(1.05 * np.eye(3), mu, lam)
    assert vm <= 1e-9 * np.abs(s).max()
    assert np.abs(s[3:]).max() <= 1e-12 * np.abs(s).max()


def test_small_simple_shear_is_linear_elastic(oracle_lib):
    mu, lam = oracle_lib.lame(E0, NU0)
    g = 1e-6
    F = np.eye(3)
    F[0, 1] = g
    s, vm = oracle_lib.cauchy(F, mu, lam)
    assert abs(s[3] - mu * g) <= 1e-5 * mu * g
    assert abs(vm - np.sqrt(3.0) * mu * g) <= 1e-5 * mu * g


def test_homogeneous_deformation_gives_uniform_tet_stress(oracle_lib):
    """u = (F - I) X on every node of a block: each tet carries the closed-form
    stress of F, in input order."""
    m = W.block_mesh((2, 3, 2), (3e-3, 4e-3, 2e-3))
    s = oracle_lib.Solver(m.X, m.tets, m.fixed, E=E0, nu=NU0)
    F = np.diag([1.01, 0.98, 1.03])
    F[0, 2] = 0.02
    u = m.X @ (F - np.eye(3)).T
    sig, vm = s.tet_stress(u)
    S = closed_form(F, s.mu, s.lam)
    assert sig.shape == (m.m, 6)
    assert np.abs(sig - six(S)[None, :]).max() <= 1e-9 * np.abs(S).max()
    assert np.abs(vm - von_mises(S)).max() <= 1e-9 * np.abs(S).max()


def test_displacement_statistics_match_brute_force(oracle_lib):
    u = np.random.default_rng(2).standard_normal((137, 3)) * 1e-3
    mx, mean = oracle_lib.displacement_stats(u)
    norms = np.sqrt((u * u).sum(axis=1))
    assert abs(mx - norms.max()) <= 1e-15 and abs(mean - norms.mean()) <= 1e-15
