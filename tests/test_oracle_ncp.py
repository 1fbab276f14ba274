"""Pins of the oracle's NCP solver (Section II.B, eq. NCP): single-contact
closed forms, the NCP conditions at every solution, brute force."""
import numpy as np
import pytest

from oracle import ncp


def _random_problem(rng, nc, ndof=None):
    ndof = ndof or 3 * nc + 2
    J = rng.normal(size=(3 * nc, ndof))
    A = rng.normal(size=(ndof, ndof))
    M = A @ A.T + ndof * np.eye(ndof)
    G = J @ np.linalg.solve(M, J.T)
    g = rng.normal(size=3 * nc) * 0.1
    mu = rng.uniform(0.2, 1.2, size=nc)
    return G, g, mu


@pytest.mark.parametrize("case", ["brk", "stk", "sld"])
def test_point_mass_local_closed_form(case):
    m, mu = 2.0, 0.6
    W = np.eye(3) / m
    b = {"brk": np.array([0.3, -0.2, 0.05]),
         "stk": np.array([0.01, -0.02, -0.5]),
         "sld": np.array([0.4, -0.3, -0.2])}[case]
    lam, mode = ncp.local_solve(W, b, mu)
    if case == "brk":
        assert mode == ncp.BRK and np.all(lam == 0)
    elif case == "stk":
        assert mode == ncp.STK
        assert np.allclose(lam, -m * b, atol=1e-14)
    else:
        assert mode == ncp.SLD
        ln = -m * b[2]
        u = b[:2] / np.linalg.norm(b[:2])
        assert np.allclose(lam, np.r_[-mu * ln * u, ln], atol=1e-12)


def test_anisotropic_local_solutions_satisfy_ncp():
    rng = np.random.default_rng(0)
    for _ in range(40):
        A = rng.normal(size=(3, 3))
        W = A @ A.T + 0.2 * np.eye(3)
        b = rng.normal(size=3)
        mu = rng.uniform(0.1, 1.5)
        lam, mode = ncp.local_solve(W, b, mu)
        assert ncp.check(W, b, np.array([mu]), lam, tol=1e-9)


def test_solutions_satisfy_every_condition():
    rng = np.random.default_rng(1)
    for nc in (1, 2, 4, 8):
        for _ in range(5):
            G, g, mu = _random_problem(rng, nc)
            lam, info = ncp.solve(G, g, mu)
            assert info["ok"]
            assert ncp.check(G, g, mu, lam, tol=1e-10)
            assert ncp.natural_residual(G, g, mu, lam).max() <= 1e-10 * max(1e-12, np.abs(lam).max())


def test_agrees_with_brute_force_enumeration():
    rng = np.random.default_rng(2)
    checked = 0
    for trial in range(30):
        nc = 1 + trial % 3
        G, g, mu = _random_problem(rng, nc)
        lam, info = ncp.solve(G, g, mu)
        sols = ncp.enumerate_solutions(G, g, mu)
        assert sols, "brute force found no solution"
        assert any(np.linalg.norm(lam - s) <= 1e-8 * max(1e-12, np.linalg.norm(s)) + 1e-14
                   for s in sols)
        checked += 1
    assert checked == 30


def test_modes_of_constructed_solution():
    # one contact of each kind on a decoupled (block-diagonal) problem
    m = 1.0
    G = np.eye(9) / m
    g = np.array([0.1, 0.0, 0.2,      # separating -> brk
                  0.01, 0.0, -0.5,    # small slip  -> stk
                  0.5, 0.2, -0.3])    # large slip  -> sld
    mu = np.array([0.5, 0.5, 0.5])
    lam, info = ncp.solve(G, g, mu)
    modes, margin = ncp.classify(G, g, mu, lam)
    assert modes == [ncp.BRK, ncp.STK, ncp.SLD]
    assert margin > 0
