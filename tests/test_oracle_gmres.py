"""Pins of the oracle's restarted GMRES (the iterative use of the product that
closes Sec. 5.3; Saad & Schultz's minimal-residual method), against facts of
the method rather than its own formulas:

* the solution of a nonsingular dense system agrees with LAPACK's solve;
* without restarts, a diagonalisable matrix with k distinct eigenvalues is
  solved in k steps (the minimal polynomial has degree k);
* within a cycle the residual norms never increase (minimal residual);
* with an H_h matrix as the operator, the true residual of the returned x,
  recomputed with the oracle's own product, meets the tolerance."""
import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O


def test_dense_system_matches_lapack():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((80, 80)) + 12.0 * np.eye(80)
    b = rng.standard_normal(80)
    x, it, hist = O.gmres(lambda v: A @ v, b, rtol=1e-13, restart=15, max_iter=400)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert hist[-1] <= 1e-13 and it <= 400


@pytest.mark.parametrize("k", [1, 3, 6])
def test_k_distinct_eigenvalues_take_k_steps(k):
    rng = np.random.default_rng(k)
    lam = np.repeat(np.arange(1.0, k + 1.0), 12)
    Q, _ = np.linalg.qr(rng.standard_normal((lam.size, lam.size)))
    A = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(lam.size)
    x, it, _ = O.gmres(lambda v: A @ v, b, rtol=1e-11, restart=lam.size, max_iter=lam.size)
    assert it == k
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_residuals_do_not_increase_within_a_cycle():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((60, 60)) + 4.0 * np.eye(60)
    b = rng.standard_normal(60)
    _, it, hist = O.gmres(lambda v: A @ v, b, rtol=1e-12, restart=60, max_iter=60)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 2))


def test_hh_operator_true_residual():
    rng = np.random.default_rng(3)
    P = rng.random((1500, 3))
    hm = O.build(P, O.Kernel(W.GAUSS, h=0.1), 1e-8, np.sqrt(3.0), -1, 64)
    shift = 0.1
    b = rng.standard_normal(1500)
    op = lambda v: O.matvec(hm, v) + shift * v
    x, it, hist = O.gmres(op, b, rtol=1e-10, restart=30, max_iter=500)
    assert np.linalg.norm(b - op(x)) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    assert hist[-1] <= 1e-10
