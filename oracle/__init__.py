"""FP64 CPU oracle for the MAID hot path -- TEST INFRASTRUCTURE ONLY.

A plain double-precision C implementation of what the HIP library computes
(the ADP-beta problem of Eq. 2.5 with a 2D convolution operator and smoothed
TV, Algorithm 1 and Algorithm 2 of arXiv 2502.09758), wrapped with ctypes for
numpy arrays.  Only ``tests/``, the package's ``smoke()`` entry and
``bench.py``'s CPU-baseline leg may import this module; the product path never
does.  It shares no code with the HIP library: its own C source, its own
header, its own struct definitions below.

Which parts are pinned, and by what, is listed per function; every function
here is pinned by a test in ``tests/test_oracle_*.py`` against something other
than itself (adjoint identities, closed forms, dense linear algebra, finite
differences, brute force), except the free-running MAID trajectory, which is
parity unpinned beyond the invariants of Lemma 1 and the schedule arithmetic
of Algorithm 2.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maid_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, MAXITER, ACCURACY_FLOOR, EINVAL, NOT_SPD = 0, 1, 2, -1, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class om_problem(ct.Structure):
    _fields_ = [("C", ct.c_int32), ("H", ct.c_int32), ("W", ct.c_int32), ("K", ct.c_int32),
                ("periodic", ct.c_int32), ("reg", ct.c_int32), ("kc", ct.c_int32),
                ("alpha", ct.c_double), ("eps_tv", ct.c_double), ("beta", ct.c_double),
                ("h1_w0", ct.c_double)]


class om_solve_info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("backtracks", ct.c_int32), ("status", ct.c_int32),
                ("res_norm", ct.c_double), ("obj", ct.c_double), ("L", ct.c_double)]


class om_hparams(ct.Structure):
    _fields_ = [("rho_lo", ct.c_double), ("rho_hi", ct.c_double), ("nu_lo", ct.c_double),
                ("nu_hi", ct.c_double), ("lambda_", ct.c_double), ("mu", ct.c_double),
                ("L_g", ct.c_double), ("eps_min", ct.c_double),
                ("max_bt", ct.c_int32), ("max_lower_iter", ct.c_int32), ("max_cg_iter", ct.c_int32)]


class om_state(ct.Structure):
    _fields_ = [("theta", ct.POINTER(ct.c_double)), ("x", ct.POINTER(ct.c_double)),
                ("q", ct.POINTER(ct.c_double)), ("eps", ct.c_double), ("delta", ct.c_double),
                ("step", ct.c_double), ("L", ct.c_double), ("k", ct.c_int32)]


class om_step_info(ct.Structure):
    _fields_ = [("accepted", ct.c_int32), ("trials", ct.c_int32), ("retries", ct.c_int32),
                ("lower_iters", ct.c_int32), ("cg_iters", ct.c_int32), ("status", ct.c_int32),
                ("psi", ct.c_double), ("ell_k", ct.c_double), ("ell_next", ct.c_double),
                ("znorm", ct.c_double), ("lower_status", ct.c_int32), ("cg_status", ct.c_int32)]


class om_trace(ct.Structure):
    _fields_ = [("replay", ct.POINTER(ct.c_int32)), ("n_replay", ct.c_int32),
                ("words", ct.POINTER(ct.c_int32)), ("values", ct.POINTER(ct.c_double)),
                ("cap_words", ct.c_int32), ("cap_values", ct.c_int32),
                ("n_words", ct.c_int32), ("n_values", ct.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ct.CDLL(_LIB)
        P = ct.POINTER(om_problem)
        d = ct.POINTER(ct.c_double)
        i32p = ct.POINTER(ct.c_int32)
        i64p = ct.POINTER(ct.c_int64)
        sig = {
            "oracle_conv": [P, d, d, d], "oracle_conv_adj": [P, d, d, d],
            "oracle_diff": [P, d, d, d], "oracle_diff_adj": [P, d, d, d],
            "oracle_reg_grad": [P, d, d], "oracle_reg_hvp": [P, d, d, d],
            "oracle_h_grad": [P, d, d, d, d], "oracle_h_hvp": [P, d, d, d, d],
            "oracle_sobolev_grad": [P, d, d, d],
            "oracle_upper_value_grad": [P, d, d, d, d, d, d],
            "oracle_hypergrad": [P, d, d, d, d, d, ct.c_int32, d, d],
            "oracle_h_grad_at": [P, d, d, d, i64p, ct.c_int64, d],
            "oracle_h_hvp_at": [P, d, d, d, i64p, ct.c_int64, d],
            "oracle_conv_at": [P, d, d, i64p, ct.c_int64, d],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None
        for name, args in {"oracle_reg_value": [P, d], "oracle_h_value": [P, d, d, d],
                           "oracle_sobolev_value": [P, d, d]}.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ct.c_double
        L.oracle_lower_solve.argtypes = [P, d, d, d, ct.c_double, ct.c_int32, d,
                                         ct.POINTER(om_solve_info), i32p, i32p]
        L.oracle_lower_solve.restype = ct.c_int
        L.oracle_adjoint_solve.argtypes = [P, d, d, d, d, ct.c_double, ct.c_int32,
                                           ct.POINTER(om_solve_info), d]
        L.oracle_adjoint_solve.restype = ct.c_int
        L.oracle_maid_step.argtypes = [P, d, d, ct.POINTER(om_state), ct.POINTER(om_hparams),
                                       ct.POINTER(om_step_info)]
        L.oracle_maid_step.restype = ct.c_int
        L.oracle_maid_step_traced.argtypes = [P, d, d, ct.POINTER(om_state), ct.POINTER(om_hparams),
                                              ct.POINTER(om_step_info), ct.POINTER(om_trace)]
        L.oracle_maid_step_traced.restype = ct.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ct.c_int
        L.oracle_set_num_threads.argtypes = [ct.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


# ----------------------------------------------------------------------------
# numpy front end
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    C: int
    H: int
    W: int
    K: int
    alpha: float = 1e-3
    eps_tv: float = 1e-2
    beta: float = 0.0
    h1_w0: float = 1.0
    periodic: bool = False
    reg: int = 0          # 0 vectorial TV, 1 channelwise TV, 2 quadratic 1/2||Dx||^2
    kc: int = 1           # kernel channels: 1 one shared KxK kernel, C one kernel per channel

    def __post_init__(self):
        if self.kc not in (1, self.C):
            raise ValueError(f"kc must be 1 or C = {self.C}, got {self.kc}")

    def c(self) -> om_problem:
        return om_problem(self.C, self.H, self.W, self.K, int(self.periodic), int(self.reg), int(self.kc),
                          float(self.alpha), float(self.eps_tv), float(self.beta), float(self.h1_w0))

    @property
    def tshape(self):
        """shape of theta and a: (K, K) shared, (C, K, K) per channel"""
        return (self.K, self.K) if self.kc == 1 else (self.kc, self.K, self.K)

    @property
    def shape(self):
        return (self.C, self.H, self.W)

    @property
    def N(self):
        return self.C * self.H * self.W

    @staticmethod
    def of(inst, **kw) -> "Problem":
        p = dict(C=inst.C, H=inst.H, W=inst.W, K=inst.K, alpha=inst.alpha, eps_tv=inst.eps_tv,
                 beta=inst.beta)
        p.update(kw)
        return Problem(**p)


def _d(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        assert a.shape == tuple(shape), (a.shape, shape)
    return a


def conv(p: Problem, th, x):
    th, x = _f64(th, p.tshape), _f64(x, p.shape)
    out = np.empty(p.shape)
    lib().oracle_conv(ct.byref(p.c()), _d(th), _d(x), _d(out))
    return out


def conv_adj(p: Problem, th, r):
    th, r = _f64(th, p.tshape), _f64(r, p.shape)
    out = np.empty(p.shape)
    lib().oracle_conv_adj(ct.byref(p.c()), _d(th), _d(r), _d(out))
    return out


def diff(p: Problem, x):
    x = _f64(x, p.shape)
    dh, dv = np.empty(p.shape), np.empty(p.shape)
    lib().oracle_diff(ct.byref(p.c()), _d(x), _d(dh), _d(dv))
    return dh, dv


def diff_adj(p: Problem, ph, pv):
    ph, pv = _f64(ph, p.shape), _f64(pv, p.shape)
    out = np.empty(p.shape)
    lib().oracle_diff_adj(ct.byref(p.c()), _d(ph), _d(pv), _d(out))
    return out


def reg_value(p: Problem, x):
    return lib().oracle_reg_value(ct.byref(p.c()), _d(_f64(x, p.shape)))


def reg_grad(p: Problem, x):
    out = np.empty(p.shape)
    lib().oracle_reg_grad(ct.byref(p.c()), _d(_f64(x, p.shape)), _d(out))
    return out


def reg_hvp(p: Problem, x, d):
    out = np.empty(p.shape)
    lib().oracle_reg_hvp(ct.byref(p.c()), _d(_f64(x, p.shape)), _d(_f64(d, p.shape)), _d(out))
    return out


def h_value(p: Problem, th, y, x):
    return lib().oracle_h_value(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(y, p.shape)),
                                _d(_f64(x, p.shape)))


def h_grad(p: Problem, th, y, x):
    out = np.empty(p.shape)
    lib().oracle_h_grad(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(y, p.shape)),
                        _d(_f64(x, p.shape)), _d(out))
    return out


def h_hvp(p: Problem, th, x, d):
    out = np.empty(p.shape)
    lib().oracle_h_hvp(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(x, p.shape)),
                       _d(_f64(d, p.shape)), _d(out))
    return out


def sobolev_value(p: Problem, th, a):
    return lib().oracle_sobolev_value(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(a, p.tshape)))


def sobolev_grad(p: Problem, th, a):
    out = np.empty(p.tshape)
    lib().oracle_sobolev_grad(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(a, p.tshape)), _d(out))
    return out


def lower_solve(p: Problem, th, y, x0, tol, max_iter=300, L=0.0, replay_bt=None):
    """FISTA with backtracking; returns (x_tilde, info dict, per-iteration
    backtrack counts).  With `replay_bt`, runs exactly `max_iter` iterations
    following the given rejection counts."""
    x = _f64(x0, p.shape).copy()
    Lc = ct.c_double(L)
    info = om_solve_info()
    trace = np.zeros(max(max_iter, 1), dtype=np.int32)
    rp = None
    if replay_bt is not None:
        rb = np.zeros(max(max_iter, 1), dtype=np.int32)
        rb[:len(replay_bt)] = np.asarray(replay_bt, dtype=np.int32)[:max_iter]
        rp = rb.ctypes.data_as(ct.POINTER(ct.c_int32))
    st = lib().oracle_lower_solve(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(y, p.shape)),
                                  _d(x), float(tol), int(max_iter), ct.byref(Lc), ct.byref(info),
                                  rp, trace.ctypes.data_as(ct.POINTER(ct.c_int32)))
    d = dict(status=st, iters=info.iters, backtracks=info.backtracks, res_norm=info.res_norm,
             obj=info.obj, L=info.L)
    return x, d, trace[:info.iters].copy()


def upper_value_grad(p: Problem, a, y, x):
    g = ct.c_double()
    gn = ct.c_double()
    grad = np.empty(p.shape)
    lib().oracle_upper_value_grad(ct.byref(p.c()), _d(_f64(a, p.tshape)), _d(_f64(y, p.shape)),
                                  _d(_f64(x, p.shape)), _d(grad), ct.byref(g), ct.byref(gn))
    return grad, g.value, gn.value


def adjoint_solve(p: Problem, th, xt, rhs, q0=None, tol=1e-2, max_iter=1000):
    q = np.zeros(p.shape) if q0 is None else _f64(q0, p.shape).copy()
    info = om_solve_info()
    tr = ct.c_double()
    st = lib().oracle_adjoint_solve(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(xt, p.shape)),
                                    _d(_f64(rhs, p.shape)), _d(q), float(tol), int(max_iter),
                                    ct.byref(info), ct.byref(tr))
    return q, dict(status=st, iters=info.iters, res_norm=info.res_norm, true_res=tr.value)


def hypergrad(p: Problem, th, a, y, xt, q, with_r=True):
    z = np.empty(p.tshape)
    zn = ct.c_double()
    a_ptr = _d(_f64(a, p.tshape)) if a is not None else None
    lib().oracle_hypergrad(ct.byref(p.c()), _d(_f64(th, p.tshape)), a_ptr, _d(_f64(y, p.shape)),
                           _d(_f64(xt, p.shape)), _d(_f64(q, p.shape)), int(bool(with_r)), _d(z),
                           ct.byref(zn))
    return z, zn.value


DEFAULT_HPARAMS = dict(rho_lo=0.5, rho_hi=1.1, nu_lo=0.5, nu_hi=1.25, lambda_=1e-4, mu=1.0,
                       L_g=0.0, eps_min=1e-12, max_bt=3, max_lower_iter=300, max_cg_iter=1000)


class MaidState:
    """Host-side MAID state (theta, warm x and q, accuracies, step size)."""

    def __init__(self, theta, x, q, eps=1e-2, delta=1e-2, step=0.1, L=0.0, k=0):
        self.theta = _f64(theta).copy()
        self.x = _f64(x).copy()
        self.q = _f64(q).copy()
        self.eps, self.delta, self.step, self.L, self.k = eps, delta, step, L, k


def maid_step(p: Problem, a, y, state: MaidState, **hp):
    h = dict(DEFAULT_HPARAMS)
    h.update(hp)
    hpc = om_hparams(**h)
    st = om_state(_d(state.theta), _d(state.x), _d(state.q), state.eps, state.delta, state.step,
                  state.L, state.k)
    info = om_step_info()
    rc = lib().oracle_maid_step(ct.byref(p.c()), _d(_f64(a, p.tshape)), _d(_f64(y, p.shape)),
                                ct.byref(st), ct.byref(hpc), ct.byref(info))
    state.eps, state.delta, state.step, state.L, state.k = st.eps, st.delta, st.step, st.L, st.k
    return rc, {f: getattr(info, f) for f, _ in om_step_info._fields_}


def maid_step_traced(p: Problem, a, y, state: MaidState, replay=None, cap=1 << 20, **hp):
    """One Algorithm 2 step with its decision trace (record layout in
    maid_oracle.h).  replay: None (free-running, the oracle's own decisions)
    or the words of a trace to follow.  Returns (rc, info, words, values):
    the trace written by this step (with the oracle's own values)."""
    h = dict(DEFAULT_HPARAMS)
    h.update(hp)
    hpc = om_hparams(**h)
    st = om_state(_d(state.theta), _d(state.x), _d(state.q), state.eps, state.delta, state.step,
                  state.L, state.k)
    info = om_step_info()
    words = np.zeros(cap, dtype=np.int32)
    values = np.zeros(cap, dtype=np.float64)
    tr = om_trace(None, 0, words.ctypes.data_as(ct.POINTER(ct.c_int32)), _d(values), cap, cap, 0, 0)
    if replay is not None:
        rp = np.ascontiguousarray(replay, dtype=np.int32)
        tr.replay = rp.ctypes.data_as(ct.POINTER(ct.c_int32))
        tr.n_replay = len(rp)
    rc = lib().oracle_maid_step_traced(ct.byref(p.c()), _d(_f64(a, p.tshape)), _d(_f64(y, p.shape)),
                                       ct.byref(st), ct.byref(hpc), ct.byref(info), ct.byref(tr))
    state.eps, state.delta, state.step, state.L, state.k = st.eps, st.delta, st.step, st.L, st.k
    return (rc, {f: getattr(info, f) for f, _ in om_step_info._fields_},
            words[:tr.n_words].copy(), values[:tr.n_values].copy())


TRACE_RECORD_VALUES = {1: 2, 2: 3, 3: 1, 4: 1, 5: 1}


def split_trace(words, values):
    """Split a decision trace into records: a list of (words, values)
    tuples, one per solve, evaluation or test, in order."""
    out, wi, vi = [], 0, 0
    words = list(words)
    while wi < len(words):
        kind = words[wi]
        if kind == 1:
            n = 4 + words[wi + 2]
        elif kind == 2:
            n = 2
        elif kind == 3:
            n = 3
        elif kind == 4:
            n = 1
        elif kind == 5:
            n = 2
        else:
            raise ValueError(f"bad trace record kind {kind} at word {wi}")
        nv = TRACE_RECORD_VALUES[kind]
        out.append((words[wi:wi + n], list(values[vi:vi + nv])))
        wi += n
        vi += nv
    return out


def _idx(idx):
    return np.ascontiguousarray(idx, dtype=np.int64)


def h_grad_at(p: Problem, th, y, x, idx):
    idx = _idx(idx)
    out = np.empty(len(idx))
    lib().oracle_h_grad_at(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(y, p.shape)),
                           _d(_f64(x, p.shape)), idx.ctypes.data_as(ct.POINTER(ct.c_int64)),
                           len(idx), _d(out))
    return out


def h_hvp_at(p: Problem, th, x, d, idx):
    idx = _idx(idx)
    out = np.empty(len(idx))
    lib().oracle_h_hvp_at(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(x, p.shape)),
                          _d(_f64(d, p.shape)), idx.ctypes.data_as(ct.POINTER(ct.c_int64)),
                          len(idx), _d(out))
    return out


def conv_at(p: Problem, th, x, idx):
    idx = _idx(idx)
    out = np.empty(len(idx))
    lib().oracle_conv_at(ct.byref(p.c()), _d(_f64(th, p.tshape)), _d(_f64(x, p.shape)),
                         idx.ctypes.data_as(ct.POINTER(ct.c_int64)), len(idx), _d(out))
    return out


# ----------------------------------------------------------------------------
# Section 4.1's baselines on the 2D problem (ADP-IFT, ADP-LISTA).  Pinned in
# tests/test_oracle_adp.py: the fixed-step iteration against its Fourier
# closed form and against a torch autograd iteration; the LISTA gradient
# against torch autograd through the unrolled iterations and against central
# differences of the unrolled loss; the IFT step against the dense
# implicit-function route.
# ----------------------------------------------------------------------------
def gd_solve(p: Problem, th, y, x0, step, n_iter):
    """The baselines' lower-level iteration: proximal gradient with a fixed
    step; the smooth regulariser's proximal map is the identity, so
    x_{k+1} = x_k - step grad_x h(x_k; theta) (Proposition 1's gradient),
    n_iter times.  Returns (x_n, [x_0, ..., x_{n-1}])."""
    x = _f64(x0, p.shape).copy()
    xs = []
    for _ in range(int(n_iter)):
        xs.append(x.copy())
        x = x - step * h_grad(p, th, y, x)
    return x, xs


def ift_step(p: Problem, a, y, theta, x0, q0, n_lower, lam_x, cg_tol, max_cg, step):
    """One ADP-IFT upper iteration: n_lower fixed-step iterations from x0, the
    implicit-function hypergradient there (CG on Algorithm 1's Hessian system
    from q0 to ||r|| <= cg_tol ||grad g||, then Eq. 3.2 with the Sobolev
    term), and theta - step z.  Returns a dict (theta, x, q, z, loss =
    g(x) + r(theta) before the step, cg_iters)."""
    x, _ = gd_solve(p, theta, y, x0, lam_x, n_lower)
    grad, g, gn = upper_value_grad(p, a, y, x)
    loss = g + sobolev_value(p, theta, a)
    q, ci = adjoint_solve(p, theta, x, grad, q0=q0, tol=cg_tol * gn, max_iter=max_cg)
    z, _ = hypergrad(p, theta, a, y, x, q, with_r=True)
    return dict(theta=_f64(theta) - step * z, x=x, q=q, z=z, loss=loss, cg_iters=ci["iters"])


def lista_grad(p: Problem, a, y, theta, x0, n_unroll, lam_x):
    """ADP-LISTA's gradient: F(theta) = g(x_n) + r(theta), x_n the n_unroll
    fixed-step iterations from x0 (held fixed), differentiated in reverse
    through the iterations.  With w = dF/dx_{k+1}, the step
    x_{k+1} = x_k - lam grad_x h(x_k; theta) adds
    -lam (d grad_x h(x_k) / d theta)^T w = lam z(x_k, w) to dF/dtheta (z the
    correlation of Eq. 3.2 without r) and passes w - lam H(x_k) w back to
    x_k; w starts at grad g(x_n).  Returns (dF/dtheta, F, x_n)."""
    x, xs = gd_solve(p, theta, y, x0, lam_x, n_unroll)
    w, g, _ = upper_value_grad(p, a, y, x)
    loss = g + sobolev_value(p, theta, a)
    dth = sobolev_grad(p, theta, a)
    for k in range(int(n_unroll) - 1, -1, -1):
        z, _ = hypergrad(p, theta, None, y, xs[k], w, with_r=False)
        dth = dth + lam_x * z
        w = w - lam_x * h_hvp(p, theta, xs[k], w)
    return dth, loss, x
