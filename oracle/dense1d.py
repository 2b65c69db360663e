"""FP64 CPU oracle for Section 4.1's 1D problem -- TEST INFRASTRUCTURE ONLY.

ADP-beta (Eq. 2.5) with beta = 0, as in Section 4.1, on a signal of n
samples whose forward operator is a full n x n matrix: the upper level
learns the matrix B of the lower level,
    upper:  min_B  g(xhat(B)) = 1/2 ||A xhat(B) - y||^2,
    lower:  xhat(B) = argmin_x  h(x; B) = 1/2 ||B x - y||^2 + alpha1 ||x||_1 + alpha2 ||x||_2^2
(the elastic-net regulariser of Section 4.1; A the known blur matrix).
The lower level is solved by proximal gradient with a fixed step (Section
4.1); the implicit-function adjoint is taken on the support of the solution,
where the lower level is smooth; Algorithm 2 runs on B.  Plain numpy, no
blocking, written from the definitions.  Only tests/ and bench.py's CPU leg
use it; it shares nothing with the HIP library.

Pinned in tests/test_oracle_dense1d.py against: the closed form for a
diagonal B; the elastic net's optimality conditions; a LAPACK solve of the
support system; central differences of F(B) with tight solves and a dense
implicit-function route; Lemma 1's decrease for accepted MAID steps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

OK, MAXITER, ACCURACY_FLOOR = 0, 1, 2


@dataclass
class Problem1D:
    n: int
    alpha1: float = 1.2e-3
    alpha2: float = 4e-3


def soft(v, t):
    """The proximal map of t ||.||_1 (soft threshold)."""
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def lower_value(p: Problem1D, B, y, x):
    r = B @ x - y
    return 0.5 * float(r @ r) + p.alpha1 * float(np.abs(x).sum()) + p.alpha2 * float(x @ x)


def prox_step(p: Problem1D, B, y, x, lam):
    """One proximal-gradient step on h: the smooth part 1/2||Bx-y||^2 +
    alpha2 ||x||^2 by a gradient step, alpha1 ||x||_1 by its proximal map."""
    grad = B.T @ (B @ x - y) + 2.0 * p.alpha2 * x
    return soft(x - lam * grad, lam * p.alpha1)


def lower_solve(p: Problem1D, B, y, x0, lam, tol, max_iter):
    """Proximal gradient with the fixed step lam; the stop test is on the
    proximal-gradient mapping G(x) = (x - prox_step(x)) / lam, the nonsmooth
    analogue of Algorithm 1's gradient test: return x once ||G(x)|| <= tol.
    Returns (x, dict(status, iters, res_norm))."""
    x = np.array(x0, dtype=np.float64, copy=True)
    for k in range(int(max_iter) + 1):
        xp = prox_step(p, B, y, x, lam)
        res = float(np.linalg.norm(x - xp)) / lam
        if res <= tol:
            return x, dict(status=OK, iters=k, res_norm=res)
        if k == max_iter:
            return x, dict(status=MAXITER, iters=k, res_norm=res)
        x = xp


def upper_value_grad(A, y, x):
    r = A @ x - y
    return A.T @ r, 0.5 * float(r @ r)


def support(x):
    return x != 0.0


def adjoint_solve(p: Problem1D, B, x, rhs, q0=None, tol=1e-10, max_iter=1000):
    """Conjugate gradients on the implicit-function system restricted to the
    support S of x, where h is twice differentiable:
    (B^T B + 2 alpha2 I)_SS q_S = rhs_S, q = 0 off S.  Stops at
    ||r|| <= tol (recursive residual)."""
    S = support(x)
    q = np.zeros_like(x) if q0 is None else np.where(S, q0, 0.0)

    def H(v):
        return np.where(S, B.T @ (B @ v) + 2.0 * p.alpha2 * v, 0.0)

    r = np.where(S, rhs, 0.0) - H(q)
    pdir = r.copy()
    gam = float(r @ r)
    it = 0
    while np.sqrt(gam) > tol and it < max_iter:
        hp = H(pdir)
        a = gam / float(pdir @ hp)
        q = q + a * pdir
        r = r - a * hp
        g2 = float(r @ r)
        pdir = r + (g2 / gam) * pdir
        gam = g2
        it += 1
    return q, dict(status=OK if np.sqrt(gam) <= tol else MAXITER, iters=it, res_norm=float(np.sqrt(gam)))


def hypergrad(B, y, x, q):
    """z = -(d (grad_x h)/dB)^T q with q supported on S: differentiating
    q^T B^T (B x - y) in B gives (B x - y) q^T + (B q) x^T."""
    return -(np.outer(B @ x - y, q) + np.outer(B @ q, x))


def lipschitz_bound(A):
    """An upper bound of ||A||_2^2, the Lipschitz constant of grad g:
    ||A||_1 ||A||_inf."""
    return float(np.abs(A).sum(axis=0).max() * np.abs(A).sum(axis=1).max())


DEFAULT_HPARAMS = dict(rho_lo=0.5, rho_hi=1.1, nu_lo=0.5, nu_hi=1.25, lambda_=1e-4, mu=1.0, eps_min=1e-12, max_bt=3,
                       max_lower_iter=300, max_cg_iter=1000, lam_x=0.1)


class State1D:
    def __init__(self, B, x, q, eps=1e-2, delta=1e-2, step=0.1, k=0):
        self.B = np.array(B, dtype=np.float64, copy=True)
        self.x = np.array(x, dtype=np.float64, copy=True)
        self.q = np.array(q, dtype=np.float64, copy=True)
        self.eps, self.delta, self.step, self.k = eps, delta, step, k


def maid_step(p: Problem1D, A, y, st: State1D, **hp):
    """One outer iteration of Algorithm 2 on B, with Eq. (3.4)'s test
    psi = l(u') + ||grad g(u')|| e + L/2 e^2 - l(u_k) + ||grad g(u_k)|| e + lambda s ||z||^2
    (l = g since beta = 0, L = lipschitz_bound(A), e = eps_k); the lower
    level by lower_solve with the fixed step lam_x.  Returns (code, info)."""
    h = dict(DEFAULT_HPARAMS)
    h.update(hp)
    Lg = lipschitz_bound(A)
    info = dict(accepted=0, trials=0, retries=0, lower_iters=0, cg_iters=0, psi=0.0, ell_k=0.0, ell_next=0.0,
                znorm=0.0)
    j = h["max_bt"]
    x = st.x.copy()
    q = st.q.copy()
    while True:
        x, li = lower_solve(p, st.B, y, x, h["lam_x"], st.eps * h["mu"], h["max_lower_iter"])
        info["lower_iters"] += li["iters"]
        G, g_k = upper_value_grad(A, y, x)
        n_k = float(np.linalg.norm(G))
        q, ci = adjoint_solve(p, st.B, x, G, q, st.delta, h["max_cg_iter"])
        info["cg_iters"] += ci["iters"]
        z = hypergrad(st.B, y, x, q)
        zn = float(np.linalg.norm(z))
        info["ell_k"], info["znorm"] = g_k, zn
        accepted = False
        for _ in range(j):
            B2 = st.B - st.step * z
            xs, li = lower_solve(p, B2, y, x, h["lam_x"], st.eps * h["mu"], h["max_lower_iter"])
            info["lower_iters"] += li["iters"]
            G2, g_n = upper_value_grad(A, y, xs)
            n_n = float(np.linalg.norm(G2))
            e = st.eps
            psi = g_n + n_n * e + 0.5 * Lg * e * e - g_k + n_k * e + h["lambda_"] * st.step * zn * zn
            info["trials"] += 1
            info["psi"], info["ell_next"] = psi, g_n
            if psi <= 0.0:
                st.B, x = B2, xs
                st.eps *= h["nu_hi"]
                st.delta *= h["nu_hi"]
                st.step *= h["rho_hi"]
                st.k += 1
                accepted = True
                break
            st.step *= h["rho_lo"]
        if accepted:
            info["accepted"] = 1
            code = OK
            break
        st.eps *= h["nu_lo"]
        st.delta *= h["nu_lo"]
        j += 1
        info["retries"] += 1
        if st.eps < h["eps_min"]:
            code = ACCURACY_FLOOR
            break
    st.x, st.q = x, q
    return code, info
