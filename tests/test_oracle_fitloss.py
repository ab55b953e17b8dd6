"""Pins of the fit-loss oracle: the normal-equation gradient form against
the residual form and against central finite differences (FP64)."""

import numpy as np
import pytest

from oracle import fitloss, tensor_ring as tr
import workloads as W


def test_gradient_forms_agree():
    cores, X = W.random_tr_problem((4, 3, 5, 2), (2, 3, 2, 2), 0, noise=0.5)
    pert = [G + 0.1 * np.random.default_rng(1).standard_normal(G.shape) for G in cores]
    a = fitloss.grad_normal_eq(X, pert)
    b = fitloss.grad_residual(X, pert)
    for x, y in zip(a, b):
        assert np.allclose(x, y, atol=1e-10 * np.abs(y).max())


def _fd_check(X, cores, n_samples, seed):
    g = fitloss.grad_normal_eq(X, cores)
    r = np.random.default_rng(seed)
    for k, G in enumerate(cores):
        for _ in range(n_samples):
            idx = tuple(r.integers(0, s) for s in G.shape)
            h = 1e-6 * max(1.0, abs(G[idx]))
            cp = [c.copy() for c in cores]
            cm = [c.copy() for c in cores]
            cp[k][idx] += h
            cm[k][idx] -= h
            fd = (fitloss.fit_loss(X, cp) - fitloss.fit_loss(X, cm)) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(g[k][idx])), (k, idx, fd, g[k][idx])


def test_finite_differences_small():
    cores, X = W.random_tr_problem((4, 3, 5, 2), (2, 3, 2, 2), 3, noise=0.5)
    pert = [G + 0.2 * np.random.default_rng(4).standard_normal(G.shape) for G in cores]
    _fd_check(X, pert, 6, 5)


def test_finite_differences_c5_subinstance():
    """The 8 x 8 x 8 x 4 corner of the c5 recipe at ranks 16."""
    w = W.make("c5", dims=(8, 8, 8), T=4)
    point = W.c5_point(w)
    _fd_check(w.X, point, 5, 6)


def test_loss_zero_at_exact_cores():
    cores, X = W.random_tr_problem((3, 4, 5), (2, 2, 3), 8)
    assert fitloss.fit_loss(X, cores) < 1e-20 * np.sum(X * X) + 1e-24
    for g in fitloss.grad_normal_eq(X, cores):
        assert np.abs(g).max() < 1e-9
