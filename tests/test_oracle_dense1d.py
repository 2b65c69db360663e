"""Pins of the 1D oracle (Section 4.1's problem; CPU only).

  lower_solve:   a diagonal B has the closed-form minimiser
                 x_i = S_alpha1(b_i y_i) / (b_i^2 + 2 alpha2); a full B's
                 result meets the elastic net's optimality conditions
                 (checked from their definition, not from the iteration);
  adjoint_solve: a LAPACK solve of the support system, and zero off the
                 support;
  hypergrad:     central differences of F(B) = g(xhat(B)) with tight solves
                 on random unit directions in R^{n x n} (the support is
                 stable under the perturbation), and the dense
                 implicit-function route dF/dB = -sum_k q_k d(grad_S h)_k/dB
                 formed entry by entry;
  maid_step:     an accepted step decreases F computed with tight solves by
                 at least lambda * step * ||z||^2 (Lemma 1) when the
                 inexact quantities are accurate enough.
"""
import numpy as np
import pytest

from oracle import dense1d as D
from paper_2502_09758_amd import synth


def small(n=40, seed=3):
    s = synth.make_1d(n=n, seed=seed, pieces=5)
    p = D.Problem1D(n, alpha1=s.alpha1, alpha2=s.alpha2)
    return s, p


def test_lower_solve_diagonal_closed_form():
    n = 30
    rng = np.random.default_rng(1)
    b = rng.uniform(0.5, 1.5, n)
    y = rng.standard_normal(n)
    p = D.Problem1D(n, alpha1=0.3, alpha2=0.05)
    x, info = D.lower_solve(p, np.diag(b), y, np.zeros(n), 0.3, 1e-13, 100000)
    ref = D.soft(b * y, p.alpha1) / (b * b + 2 * p.alpha2)
    assert info["status"] == D.OK
    assert np.abs(x - ref).max() <= 1e-12
    assert (ref == 0).sum() > 3          # the threshold is active somewhere


def test_lower_solve_optimality_conditions():
    s, p = small()
    x, info = D.lower_solve(p, s.A, s.y, np.zeros(p.n), 0.1, 1e-12, 500000)
    assert info["status"] == D.OK
    smooth = s.A.T @ (s.A @ x - s.y) + 2 * p.alpha2 * x
    S = x != 0
    # on the support the subgradient is alpha1 sign(x); off it |smooth| <= alpha1
    assert np.abs(smooth[S] + p.alpha1 * np.sign(x[S])).max() <= 1e-10
    assert np.abs(smooth[~S]).max() <= p.alpha1 * (1 + 1e-9)
    assert 0 < S.sum() < p.n


def test_adjoint_solve_matches_lapack_on_support():
    s, p = small()
    x, _ = D.lower_solve(p, s.A, s.y, np.zeros(p.n), 0.1, 1e-12, 500000)
    rhs = np.random.default_rng(2).standard_normal(p.n)
    q, info = D.adjoint_solve(p, s.A, x, rhs, tol=1e-13, max_iter=10 * p.n)
    S = x != 0
    Hs = (s.A.T @ s.A + 2 * p.alpha2 * np.eye(p.n))[np.ix_(S, S)]
    ref = np.linalg.solve(Hs, rhs[S])
    assert info["status"] == D.OK and info["iters"] <= S.sum() + 5
    assert np.linalg.norm(q[S] - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.all(q[~S] == 0)


def _F(p, B, A, y, x0):
    x, info = D.lower_solve(p, B, y, x0, 0.1, 1e-13, 2000000)
    assert info["status"] == D.OK
    return D.upper_value_grad(A, y, x)[1], x


def test_hypergrad_central_differences_and_dense_route():
    s, p = small(n=24, seed=5)
    B = s.A + 0.01 * np.random.default_rng(4).standard_normal(s.A.shape)
    F0, x = _F(p, B, s.A, s.y, np.zeros(p.n))
    G, _ = D.upper_value_grad(s.A, s.y, x)
    q, _ = D.adjoint_solve(p, B, x, G, tol=1e-14, max_iter=10 * p.n)
    z = D.hypergrad(B, s.y, x, q)
    # dense route: d(grad_S h)_k / dB_ij for every (k in S, i, j), contracted with q
    S = np.flatnonzero(x != 0)
    r = B @ x - s.y
    zd = np.zeros_like(B)
    for k in S:
        # (grad h)_k = sum_i B_ik r_i + ...; d/dB_ij = delta_jk r_i + B_ik x_j
        dk = np.zeros_like(B)
        dk[:, k] += r
        dk += np.outer(B[:, k], x)
        zd -= q[k] * dk
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    rng = np.random.default_rng(6)
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(B.shape)
        d /= np.linalg.norm(d)
        Fp, xp = _F(p, B + h * d, s.A, s.y, x)
        Fm, xm = _F(p, B - h * d, s.A, s.y, x)
        assert np.array_equal(xp != 0, x != 0) and np.array_equal(xm != 0, x != 0)
        fd = (Fp - Fm) / (2 * h)
        # z is dF/dB (Eq. 3.2: the implicit-function gradient)
        assert abs(fd - float(np.vdot(z, d))) <= 1e-6 * np.linalg.norm(z)


def test_maid_step_accepted_decrease():
    s, p = small(n=32, seed=9)
    st = D.State1D(s.A, np.zeros(p.n), np.zeros(p.n), eps=1e-7, delta=1e-8, step=0.5)
    F0, _ = _F(p, st.B, s.A, s.y, np.zeros(p.n))
    acc = 0
    for _ in range(3):
        code, info = D.maid_step(p, s.A, s.y, st, max_lower_iter=400000, max_cg_iter=4000, eps_min=1e-14)
        assert code == D.OK
        if info["accepted"]:
            acc += 1
            F1, _ = _F(p, st.B, s.A, s.y, st.x)
            assert F1 <= F0 - 1e-4 * (st.step / 1.1) * info["znorm"] ** 2 * 0.999
            F0 = F1
    assert acc >= 2
