"""Pins of the oracle's MAID step (Algorithm 2 with psi of Eq. 3.4), CPU only.

  - Lemma 1 (sufficient decrease): with mu certified as a lower bound of the
    lower-level Hessian (smallest eigenvalue of K^T K, since the TV Hessian is
    positive semi-definite), every accepted step decreases the exact F(theta)
    = g(xhat(theta)) + r(theta), computed by dense Newton solves, by at least
    lambda * s * ||z||^2;
  - the schedule arithmetic of Algorithm 2 (accuracies and step size are
    products of the four factors);
  - the accuracy floor error path;
  - the defaults equal the hyperparameters printed in Section 4.1.
The free-running trajectory itself is parity unpinned beyond these."""
import json
import os

import numpy as np
import pytest
import scipy.signal as ss

import oracle as O
import _ref_torch as R
from paper_2502_09758_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_hparams.json")))


def test_defaults_are_the_papers():
    m = GOLD["maid"]
    d = O.DEFAULT_HPARAMS
    assert (d["rho_hi"], d["rho_lo"], d["nu_hi"], d["nu_lo"], d["max_lower_iter"]) == \
        (m["rho_hi"], m["rho_lo"], m["nu_hi"], m["nu_lo"], m["max_lower_iter"])


def _well_conditioned(H=12, W=12, C=1, seed=3):
    K = 3
    a = np.array([[0.0, 0.1, 0.0], [0.1, 0.6, 0.1], [0.0, 0.1, 0.0]])
    inst = synth.make("cfg1", H=H, W=W, C=C, K=7, seed=seed)
    true = a + 0.05 * np.array([[1, 0, -1], [0, 0, 0], [-1, 0, 1.0]])
    y = np.stack([ss.convolve2d(inst.x_true[c], true, mode="same") for c in range(C)])
    y = y + 0.01 * np.random.default_rng(seed).standard_normal(y.shape)
    p = O.Problem(C, H, W, K, alpha=2e-3, eps_tv=1e-2, beta=1e-3)
    N = H * W
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1
        A[:, k] = ss.convolve2d(e.reshape(H, W), a, mode="same").ravel()
    mu = np.linalg.eigvalsh(A.T @ A).min()
    return p, a, y, mu


def _F(p, th, a, y, x0):
    xh = R.newton_solve(R.t(th), R.t(y), R.t(x0), p.alpha, p.eps_tv)
    return float(R.g(R.t(a), R.t(y), xh) + R.sobolev(R.t(th), R.t(a), p.beta))


def test_lemma1_sufficient_decrease_with_certified_mu():
    p, a, y, mu = _well_conditioned()
    assert mu > 1e-3
    lam = 0.05
    st = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    F_prev = _F(p, st.theta, a, y, y)
    accepted = 0
    for k in range(6):
        th_before = st.theta.copy()
        s_before = st.step
        rc, info = O.maid_step(p, a, y, st, mu=mu, lambda_=lam, max_lower_iter=100000,
                               max_cg_iter=100000, eps_min=1e-6)
        if rc == O.ACCURACY_FLOOR:      # the paper's stop: accuracy driven below 1e-6
            np.testing.assert_array_equal(st.theta, th_before)
            break
        assert rc == O.OK and info["accepted"]
        accepted += 1
        assert info["psi"] <= 0.0
        # the accepted step length: s_before shrunk once per rejected trial
        s_used = s_before * 0.5 ** (info["trials"] - 1)
        F_new = _F(p, st.theta, a, y, st.x)
        assert F_new - F_prev <= -lam * s_used * info["znorm"] ** 2 * (1 - 1e-9)
        F_prev = F_new
    assert accepted >= 3


@pytest.mark.parametrize("step0,eps0", [(0.3, 1e-4), (40.0, 4e-4)])
def test_schedule_arithmetic(step0, eps0):
    p, a, y, mu = _well_conditioned()
    st = O.MaidState(a, y, np.zeros_like(y), eps=eps0, delta=2 * eps0, step=step0)
    seen = 0
    for k in range(4):
        e0, d0, s0 = st.eps, st.delta, st.step
        rc, info = O.maid_step(p, a, y, st, eps_min=1e-7, max_lower_iter=100000, max_cg_iter=100000)
        if rc == O.ACCURACY_FLOOR:
            break
        assert rc == O.OK and info["accepted"] == 1
        r, t = info["retries"], info["trials"]
        assert st.eps == pytest.approx(e0 * 0.5 ** r * 1.25, rel=1e-15)
        assert st.delta == pytest.approx(d0 * 0.5 ** r * 1.25, rel=1e-15)
        assert st.step == pytest.approx(s0 * 0.5 ** (t - 1) * 1.1, rel=1e-15)
        # trials: max_bt + (max_bt+1) + ... per failed retry, then the accepted index
        full = sum(3 + i for i in range(r))
        assert full < t <= full + 3 + r
        assert st.k == seen + 1
        assert info["psi"] <= 0
        seen += 1
    assert seen >= 2


def test_accuracy_floor():
    inst = synth.make("cfg1", H=16, W=16)
    p = O.Problem.of(inst)
    st = O.MaidState(inst.a, inst.y, np.zeros_like(inst.y), eps=1e-2, delta=1e-2, step=0.1)
    rc, info = O.maid_step(p, inst.a, inst.y, st, lambda_=1e9, eps_min=1e-3)
    assert rc == O.ACCURACY_FLOOR and info["accepted"] == 0
    np.testing.assert_array_equal(st.theta, inst.a)
    assert st.eps < 1e-3 and info["retries"] == 4


def test_solve_cap_is_flagged_not_dropped():
    """A lower-level or CG solve that stops at its iteration cap is carried on
    with and flagged: the step reports which solve kind hit its cap and
    returns MAXITER (a warning) where it would otherwise return OK."""
    p, a, y, mu = _well_conditioned()
    st = O.MaidState(a, y, np.zeros_like(y), eps=1e-6, delta=1e-6, step=0.3)
    rc, info = O.maid_step(p, a, y, st, max_lower_iter=3, eps_min=1e-9)
    assert info["lower_status"] == O.MAXITER
    assert rc in (O.MAXITER, O.ACCURACY_FLOOR)
    st = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-9, step=0.3)
    rc, info = O.maid_step(p, a, y, st, max_cg_iter=2, max_lower_iter=100000, eps_min=1e-9)
    assert info["cg_status"] == O.MAXITER and info["lower_status"] == O.OK
    assert rc in (O.MAXITER, O.ACCURACY_FLOOR)
    # uncapped: both flags clear and the step returns OK
    st = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    rc, info = O.maid_step(p, a, y, st, max_lower_iter=100000, max_cg_iter=100000, eps_min=1e-7)
    assert rc == O.OK and info["lower_status"] == O.OK and info["cg_status"] == O.OK


def test_replay_of_own_trace_is_bitwise():
    """The replay mode pinned to the free-running step: following the
    oracle's own recorded decisions reproduces its result bit for bit, with
    the same words and values."""
    p, a, y, mu = _well_conditioned(C=2, seed=4)
    s_free = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    s_rep = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    kinds = set()
    for k in range(3):
        rc, info, w, v = O.maid_step_traced(p, a, y, s_free, max_lower_iter=100000, eps_min=1e-7)
        rc2, info2, w2, v2 = O.maid_step_traced(p, a, y, s_rep, replay=w, max_lower_iter=100000, eps_min=1e-7)
        assert rc == rc2 and info == info2
        np.testing.assert_array_equal(w, w2)
        np.testing.assert_array_equal(v, v2)
        np.testing.assert_array_equal(s_free.theta, s_rep.theta)
        np.testing.assert_array_equal(s_free.x, s_rep.x)
        np.testing.assert_array_equal(s_free.q, s_rep.q)
        recs = O.split_trace(w, v)
        kinds |= {r[0][0] for r in recs}
        # the record counts agree with the step's own tallies
        assert sum(r[0][2] for r in recs if r[0][0] == 1) == info["lower_iters"]
        assert sum(r[0][1] for r in recs if r[0][0] == 3) == info["cg_iters"]
        assert sum(1 for r in recs if r[0][0] == 5) == info["trials"]
        psis = [r[1][0] for r in recs if r[0][0] == 5]
        assert psis[-1] == info["psi"] and (psis[-1] <= 0) == bool(info["accepted"])
        if rc != O.OK:
            break
    assert kinds == {1, 2, 3, 4, 5}


def test_replay_follows_foreign_decisions():
    """A replayed acceptance is taken even where the oracle's own psi says
    otherwise, and a malformed trace is an error."""
    p, a, y, mu = _well_conditioned(seed=5)
    s0 = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    rc, info, w, v = O.maid_step_traced(p, a, y, s0, max_lower_iter=100000, eps_min=1e-7)
    recs = O.split_trace(w, v)
    assert info["accepted"] == 1 and info["trials"] < 3
    # the accepted psi test turned into a rejection, followed by one more
    # trial (replaying the last trial's lower-level decisions) that accepts
    last = max(k for k, (rw, _) in enumerate(recs) if rw[0] == 5)
    trial = [rw for rw, _ in recs if rw[0] == 1 and rw[1] == 1][-1]
    out = []
    for k, (rw, _) in enumerate(recs):
        out += [5, 0] + list(trial) + [2, 1] + [5, 1] if k == last else list(rw)
    s1 = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    rc1, info1, w1, v1 = O.maid_step_traced(p, a, y, s1, replay=out, max_lower_iter=100000, eps_min=1e-7)
    assert rc1 == O.OK and info1["accepted"] == 1 and info1["trials"] == info["trials"] + 1
    assert s1.step == pytest.approx(0.3 * 0.5 ** info["trials"] * 1.1, rel=1e-15)
    np.testing.assert_array_equal(w1, out)
    s2 = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    rc2, _, _, _ = O.maid_step_traced(p, a, y, s2, replay=[1, 0, 3], eps_min=1e-7)
    assert rc2 == O.EINVAL
