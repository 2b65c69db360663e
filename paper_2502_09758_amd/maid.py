"""Torch front end of libmaid: one `Maid` context per problem shape.

Names follow the C ABI (include/maid.h) and the paper: `lower_solve` is the
lower-level solve of Algorithm 1, `adjoint_solve` its Hessian system,
`hypergrad` its last line (Eq. 3.2), `maid_step` one iteration of
Algorithm 2.  Tensors live on the GPU; this module only checks and
marshals them.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float32: L.MAID_F32, torch.float64: L.MAID_F64}

# Algorithm 2 hyperparameters; the four factors and the iteration cap are the
# values printed in Section 4.1, the rest are this build's readings.
DEFAULT_HPARAMS = dict(rho_lo=0.5, rho_hi=1.1, nu_lo=0.5, nu_hi=1.25, lambda_=1e-4, mu=1.0,
                       L_g=0.0, eps_min=1e-12, max_bt=3, max_lower_iter=300, max_cg_iter=1000)


def _ptr(t):
    return ct.c_void_p(t.data_ptr())


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class SolveInfo:
    status: int
    iters: int
    backtracks: int = 0
    res_norm: float = 0.0
    L: float = 0.0
    trace: list = field(default_factory=list)


@dataclass
class MaidState:
    """theta (K x K float64, or C x K x K with per-channel kernels), x and q
    (C x H x W, storage dtype) on the GPU,
    updated in place by `Maid.maid_step`."""
    theta: torch.Tensor
    x: torch.Tensor
    q: torch.Tensor
    eps: float = 1e-2
    delta: float = 1e-2
    step: float = 0.1
    L: float = 0.0
    k: int = 0


class Maid:
    def __init__(self, C, H, W, K, dtype=torch.float32, alpha=1e-3, eps_tv=1e-2, beta=0.0,
                 h1_w0=1.0, reg=L.MAID_REG_TV, kc=1):
        if dtype not in _DT:
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.C, self.H, self.W, self.K = int(C), int(H), int(W), int(K)
        self.kc = int(kc)          # kernel planes: 1 shared kernel, C one kernel per channel
        self.dtype = dtype
        self.alpha, self.eps_tv, self.beta, self.h1_w0, self.reg = alpha, eps_tv, beta, h1_w0, reg
        self.desc = L.maid_desc(H=self.H, W=self.W, C=self.C, K=self.K, dtype=_DT[dtype], boundary=0, reg=int(reg),
                                kc=self.kc, alpha=float(alpha), eps_tv=float(eps_tv), beta=float(beta),
                                h1_w0=float(h1_w0))
        self._h = None
        self._h = L.create(self.desc)

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and L is not None and L._lib is not None:
            L._lib.maid_destroy(ct.c_void_p(h))

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass

    # ------------------------------------------------------------------ checks
    @property
    def handle(self):
        return ct.c_void_p(self._h)

    @property
    def shape(self):
        return (self.C, self.H, self.W)

    def _img(self, t, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous {self.dtype} of shape {self.shape}, got "
                             f"{t.dtype} {tuple(t.shape)}")
        return t

    @property
    def kshape(self):
        """shape of theta, a and z: (K, K) shared, (C, K, K) per channel"""
        return (self.K, self.K) if self.kc <= 1 else (self.kc, self.K, self.K)

    def _ker(self, t, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != torch.float64 or tuple(t.shape) != self.kshape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous float64 of shape {self.kshape}")
        return t

    def _check(self, rc, what):
        if rc < 0:
            raise L.MaidError(rc, f"{what}: {L.last_error(self.handle)}")
        return rc

    def config(self) -> str:
        return L.lib().maid_config_string(self.handle).decode()

    def set_tile_rows(self, rows: int):
        self._check(L.lib().maid_set_tile_rows(self.handle, int(rows)), "set_tile_rows")

    def set_one_pass_cg(self, enable: bool):
        """Opt in to the one-pass (Chronopoulos-Gear) CG on one-pass instances."""
        self._check(L.lib().maid_set_one_pass_cg(self.handle, int(bool(enable))), "set_one_pass_cg")

    def set_mfma(self, enable: bool):
        """Large-kernel correlations on the matrix cores (FP32 storage, K >= 13,
        4 or 8 rows per thread; the default) or on the vector ALUs."""
        self._check(L.lib().maid_set_mfma(self.handle, int(bool(enable))), "set_mfma")

    def set_one_pass(self, mode: int):
        """Lower-level form where the one-pass form applies: -1 tuned or size
        rule (default), 0 two-pass, 1 one-pass."""
        self._check(L.lib().maid_set_one_pass(self.handle, int(mode)), "set_one_pass")

    def one_pass_forms(self):
        """Per instance: 1 if it runs the one-pass lower-level form."""
        n = int(L.lib().maid_batch_size(self.handle))
        out = (ct.c_int32 * max(1, n))()
        self._check(L.lib().maid_one_pass_forms(self.handle, out), "one_pass_forms")
        return [int(out[i]) for i in range(n)]

    def set_team(self, members: int):
        """Members per team of the persistent loops: -1 size rule, 0 off."""
        self._check(L.lib().maid_set_team(self.handle, int(members)), "set_team")

    def autotune(self, theta, y, probe_iters=20):
        """Pick the tile height by timing short probe solves; returns the rows
        per thread chosen."""
        self._ker(theta, "theta"), self._img(y, "y")
        th = (ct.c_void_p * 1)(theta.data_ptr())
        yy = (ct.c_void_p * 1)(y.data_ptr())
        rows = (ct.c_int32 * 1)()
        self._check(L.lib().maid_autotune(self.handle, th, yy, int(probe_iters), rows, _stream()), "autotune")
        return rows[0]

    def profile(self, enable: bool):
        """Start (reset) or stop per-launch kernel timing."""
        self._check(L.lib().maid_profile(self.handle, int(bool(enable))), "profile")

    def profile_read(self) -> dict:
        """{kernel kind: (launches, launches that did a pass of work, total milliseconds)}"""
        out = {}
        for k in range(L.PROF_KINDS):
            n, w, ms = ct.c_int64(), ct.c_int64(), ct.c_double()
            self._check(L.lib().maid_profile_read(self.handle, k, ct.byref(n), ct.byref(w), ct.byref(ms)),
                        "profile_read")
            out[L.lib().maid_profile_name(k).decode()] = (n.value, w.value, ms.value)
        return out

    # ------------------------------------------------------------------ entry points
    def lower_solve(self, theta, y, x, tol, max_iter=300, L_est=0.0, trace=False):
        """Solve the lower level in place in `x` (in: start, out: result)."""
        self._ker(theta, "theta"), self._img(y, "y"), self._img(x, "x")
        Lc = ct.c_double(L_est)
        info = L.maid_solve_info()
        tr = (ct.c_int32 * max(1, max_iter))() if trace else None
        rc = L.lib().maid_lower_solve(self.handle, _ptr(theta), _ptr(y), _ptr(x), float(tol), int(max_iter),
                                      ct.byref(Lc), ct.byref(info), tr, _stream())
        self._check(rc, "lower_solve")
        return SolveInfo(rc, info.iters, info.backtracks, info.res_norm, info.L,
                         list(tr[:info.iters]) if trace else [])

    def lower_solve_refined(self, theta, y, x, tol, max_iter=300, rel_tol=1e-7, max_newton=4, max_cg=2000,
                            L_est=0.0):
        """The precision form: lower-level solve to `tol`, then Newton steps
        (FP64 residual, CG correction in the storage type) until the relative
        step is below `rel_tol`.  Returns (SolveInfo of the first phase, dict
        of the refinement: newton_steps, cg_iters, status, rel_step,
        grad_norm)."""
        self._ker(theta, "theta"), self._img(y, "y"), self._img(x, "x")
        Lc = ct.c_double(L_est)
        info = L.maid_solve_info()
        rinfo = L.maid_refine_info()
        rc = L.lib().maid_lower_solve_refined(self.handle, _ptr(theta), _ptr(y), _ptr(x), float(tol), int(max_iter),
                                              float(rel_tol), int(max_newton), int(max_cg), ct.byref(Lc),
                                              ct.byref(info), ct.byref(rinfo), _stream())
        self._check(rc, "lower_solve_refined")
        return (SolveInfo(info.status, info.iters, info.backtracks, info.res_norm, info.L),
                {f: getattr(rinfo, f) for f, _ in L.maid_refine_info._fields_})

    def upper_value_grad(self, a, y, x, grad_out=None):
        self._ker(a, "a"), self._img(y, "y"), self._img(x, "x")
        if grad_out is not None:
            self._img(grad_out, "grad_out")
        g, gn = ct.c_double(), ct.c_double()
        rc = L.lib().maid_upper_value_grad(self.handle, _ptr(a), _ptr(y), _ptr(x),
                                           _ptr(grad_out) if grad_out is not None else None,
                                           ct.byref(g), ct.byref(gn), _stream())
        self._check(rc, "upper_value_grad")
        return g.value, gn.value

    def adjoint_solve(self, theta, x_tilde, rhs, q, tol, max_iter=1000):
        """CG on the lower-level Hessian, in place in `q`."""
        self._ker(theta, "theta"), self._img(x_tilde, "x_tilde"), self._img(rhs, "rhs"), self._img(q, "q")
        info = L.maid_solve_info()
        rc = L.lib().maid_adjoint_solve(self.handle, _ptr(theta), _ptr(x_tilde), _ptr(rhs), _ptr(q), float(tol),
                                        int(max_iter), ct.byref(info), _stream())
        self._check(rc, "adjoint_solve")
        return SolveInfo(rc, info.iters, 0, info.res_norm, 0.0)

    def hypergrad(self, theta, a, y, x_tilde, q, with_r=True, z=None):
        self._ker(theta, "theta"), self._img(y, "y"), self._img(x_tilde, "x_tilde"), self._img(q, "q")
        if a is not None:
            self._ker(a, "a")
        if z is None:
            z = torch.empty(self.kshape, dtype=torch.float64, device=theta.device)
        self._ker(z, "z")
        zn = ct.c_double()
        rc = L.lib().maid_hypergrad(self.handle, _ptr(theta), _ptr(a) if a is not None else None, _ptr(y),
                                    _ptr(x_tilde), _ptr(q), int(bool(with_r)), _ptr(z), ct.byref(zn), _stream())
        self._check(rc, "hypergrad")
        return z, zn.value

    def apply_operator(self, theta, x, out=None, adjoint=False):
        """theta * x (or the adjoint correlation theta . x)."""
        self._ker(theta, "theta"), self._img(x, "x")
        if out is None:
            out = torch.empty_like(x)
        self._img(out, "out")
        self._check(L.lib().maid_apply_operator(self.handle, _ptr(theta), _ptr(x), _ptr(out), int(bool(adjoint)),
                                                _stream()), "apply_operator")
        return out

    def sobolev_value(self, theta, a):
        self._ker(theta, "theta"), self._ker(a, "a")
        r = ct.c_double()
        self._check(L.lib().maid_sobolev_value(self.handle, _ptr(theta), _ptr(a), ct.byref(r), _stream()),
                    "sobolev_value")
        return r.value

    def maid_step(self, a, y, state: MaidState, **hp):
        self._ker(a, "a"), self._img(y, "y"), self._ker(state.theta, "theta")
        self._img(state.x, "x"), self._img(state.q, "q")
        h = dict(DEFAULT_HPARAMS)
        h.update(hp)
        hpc = L.maid_hparams(**h)
        st = L.maid_state(state.theta.data_ptr(), state.x.data_ptr(), state.q.data_ptr(), state.eps, state.delta,
                          state.step, state.L, state.k)
        info = L.maid_step_info()
        rc = L.lib().maid_step(self.handle, _ptr(a), _ptr(y), ct.byref(st), ct.byref(hpc), ct.byref(info), _stream())
        self._check(rc, "maid_step")
        state.eps, state.delta, state.step, state.L, state.k = st.eps, st.delta, st.step, st.L, st.k
        return rc, {f: getattr(info, f) for f, _ in L.maid_step_info._fields_}

    # ---------------------------------------------------------------- Section 4.1's baselines
    def gd_solve(self, theta, y, x, step, n_iter, tol=0.0, hist=None):
        """maid_gd_solve: n_iter fixed-step gradient iterations, in place in x;
        hist (optional, n_iter x C x H x W) receives x_1 .. x_n."""
        self._ker(theta, "theta"), self._img(y, "y"), self._img(x, "x")
        hp = None
        if hist is not None:
            if not isinstance(hist, torch.Tensor) or not hist.is_cuda or hist.dtype != self.dtype or \
                    not hist.is_contiguous() or hist.numel() < int(n_iter) * self.C * self.H * self.W:
                raise ValueError("hist must be a contiguous CUDA tensor of n_iter*C*H*W elements of the storage type")
            hp = hist.data_ptr()
        info = L.maid_solve_info()
        rc = L.lib().maid_gd_solve(self.handle, _ptr(theta), _ptr(y), _ptr(x), float(step), int(n_iter), float(tol),
                                   hp, ct.byref(info), _stream())
        self._check(rc, "gd_solve")
        return SolveInfo(info.status, info.iters, info.backtracks, info.res_norm, info.L)

    def hessian_apply(self, theta, x, w, out=None):
        """maid_hessian_apply: out = H(x) w (Proposition 1's Hessian)."""
        self._ker(theta, "theta"), self._img(x, "x"), self._img(w, "w")
        if out is None:
            out = torch.empty_like(w)
        self._img(out, "out")
        self._check(L.lib().maid_hessian_apply(self.handle, _ptr(theta), _ptr(x), _ptr(w), _ptr(out), _stream()),
                    "hessian_apply")
        return out

    def _adp_state(self, state: MaidState):
        return L.maid_state(state.theta.data_ptr(), state.x.data_ptr(), state.q.data_ptr(), state.eps, state.delta,
                            state.step, state.L, state.k)

    def ift_step(self, a, y, state: MaidState, n_lower=500, lambda_x=0.1, cg_tol=1e-3, max_cg=1000):
        """maid_ift_step: one ADP-IFT upper iteration (state.step is the upper
        step size); returns (rc, info dict)."""
        self._ker(a, "a"), self._img(y, "y"), self._ker(state.theta, "theta")
        self._img(state.x, "x"), self._img(state.q, "q")
        st = self._adp_state(state)
        info = L.maid_step_info()
        rc = L.lib().maid_ift_step(self.handle, _ptr(a), _ptr(y), ct.byref(st), int(n_lower), float(lambda_x),
                                   float(cg_tol), int(max_cg), ct.byref(info), _stream())
        self._check(rc, "ift_step")
        state.k = st.k
        return rc, {f: getattr(info, f) for f, _ in L.maid_step_info._fields_}

    def lista_step(self, a, y, state: MaidState, n_unroll=50, lambda_x=0.1):
        """maid_lista_step: one ADP-LISTA upper iteration; returns (rc, info
        dict).  The context must be on the two-pass form (set_one_pass(0))."""
        self._ker(a, "a"), self._img(y, "y"), self._ker(state.theta, "theta"), self._img(state.x, "x")
        if state.q is not None:
            self._img(state.q, "q")
        st = self._adp_state(state)
        info = L.maid_step_info()
        rc = L.lib().maid_lista_step(self.handle, _ptr(a), _ptr(y), ct.byref(st), int(n_unroll), float(lambda_x),
                                     ct.byref(info), _stream())
        self._check(rc, "lista_step")
        state.k = st.k
        return rc, {f: getattr(info, f) for f, _ in L.maid_step_info._fields_}

    def maid_step_traced(self, a, y, state: MaidState, cap=1 << 20, **hp):
        """maid_step with its decision trace (record layout in maid.h):
        returns (rc, info, words, values)."""
        w = (ct.c_int32 * cap)()
        v = (ct.c_double * cap)()
        self._check(L.lib().maid_set_step_trace(self.handle, 0, w, cap, v, cap), "set_step_trace")
        try:
            rc, info = self.maid_step(a, y, state, **hp)
        finally:
            nw, nv = ct.c_int32(), ct.c_int32()
            L.lib().maid_step_trace_length(self.handle, ct.byref(nw), ct.byref(nv))
            L.lib().maid_set_step_trace(self.handle, 0, None, 0, None, 0)
        return rc, info, list(w[:nw.value]), list(v[:nv.value])


class MaidBatch:
    """A ragged batch of independent instances in one context (the batched
    form of the C ABI).  `specs` is a list of dicts with keys C, H, W, K and
    optionally alpha, eps_tv, beta, h1_w0, reg; one storage dtype for all.
    Per-instance tensors are passed as lists."""

    def __init__(self, specs, dtype=torch.float32):
        if dtype not in _DT:
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.specs = [dict(alpha=1e-3, eps_tv=1e-2, beta=0.0, h1_w0=1.0, reg=L.MAID_REG_TV, kc=1) | dict(s)
                      for s in specs]
        self.n = len(self.specs)
        self.descs = [L.maid_desc(H=int(s["H"]), W=int(s["W"]), C=int(s["C"]), K=int(s["K"]), dtype=_DT[dtype],
                                  boundary=0, reg=int(s["reg"]), kc=int(s["kc"]),
                                  alpha=float(s["alpha"]), eps_tv=float(s["eps_tv"]), beta=float(s["beta"]),
                                  h1_w0=float(s["h1_w0"]))
                      for s in self.specs]
        self._h = None
        self._h = L.create_batch(self.descs)

    close = Maid.close
    __del__ = Maid.__del__
    handle = Maid.handle
    config = Maid.config
    set_tile_rows = Maid.set_tile_rows
    set_team = Maid.set_team
    set_one_pass_cg = Maid.set_one_pass_cg
    set_mfma = Maid.set_mfma
    set_one_pass = Maid.set_one_pass
    one_pass_forms = Maid.one_pass_forms
    profile = Maid.profile
    profile_read = Maid.profile_read
    _check = Maid._check

    def _imgs(self, ts, name):
        if len(ts) != self.n:
            raise ValueError(f"{name}: need {self.n} tensors")
        for i, t in enumerate(ts):
            s = self.specs[i]
            shape = (s["C"], s["H"], s["W"])
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.dtype or \
                    tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name}[{i}] must be a contiguous CUDA {self.dtype} tensor of shape {shape}")
        return (ct.c_void_p * self.n)(*[t.data_ptr() for t in ts])

    def _kers(self, ts, name):
        if len(ts) != self.n:
            raise ValueError(f"{name}: need {self.n} tensors")
        for i, t in enumerate(ts):
            ks = self._kshape(i)
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or \
                    tuple(t.shape) != ks or not t.is_contiguous():
                raise ValueError(f"{name}[{i}] must be a contiguous CUDA float64 tensor of shape {ks}")
        return (ct.c_void_p * self.n)(*[t.data_ptr() for t in ts])

    def _kshape(self, i):
        s = self.specs[i]
        return (s["K"], s["K"]) if s["kc"] <= 1 else (s["kc"], s["K"], s["K"])

    def _rc(self, rc, what):
        if rc < 0 and rc not in (L.NOT_SPD, L.NONFINITE):
            raise L.MaidError(rc, f"{what}: {L.last_error(self.handle)}")
        return rc

    def autotune(self, thetas, ys, probe_iters=20):
        """Per K group, pick the tile height by timing short probe solves;
        returns the rows per thread chosen for each instance."""
        th, y = self._kers(thetas, "theta"), self._imgs(ys, "y")
        rows = (ct.c_int32 * self.n)()
        self._check(L.lib().maid_autotune(self.handle, th, y, int(probe_iters), rows, _stream()), "autotune")
        return list(rows)

    def lower_solve(self, thetas, ys, xs, tols, max_iter=300, L_est=None):
        """Batched lower-level solve, in place in `xs`; returns (rc, [SolveInfo])."""
        th, y, x = self._kers(thetas, "theta"), self._imgs(ys, "y"), self._imgs(xs, "x")
        tol = (ct.c_double * self.n)(*[float(t) for t in tols])
        Lc = (ct.c_double * self.n)(*([0.0] * self.n if L_est is None else [float(v) for v in L_est]))
        info = (L.maid_solve_info * self.n)()
        rc = L.lib().maid_batch_lower_solve(self.handle, th, y, x, tol, int(max_iter), Lc, info, _stream())
        self._rc(rc, "batch_lower_solve")
        return rc, [SolveInfo(i.status, i.iters, i.backtracks, i.res_norm, i.L) for i in info]

    def adjoint_solve(self, thetas, xts, rhss, qs, tols, max_iter=1000):
        """Batched CG solve, in place in `qs`; returns (rc, [SolveInfo])."""
        th, xt, b, q = self._kers(thetas, "theta"), self._imgs(xts, "x_tilde"), self._imgs(rhss, "rhs"), \
            self._imgs(qs, "q")
        tol = (ct.c_double * self.n)(*[float(t) for t in tols])
        info = (L.maid_solve_info * self.n)()
        rc = L.lib().maid_batch_adjoint_solve(self.handle, th, xt, b, q, tol, int(max_iter), info, _stream())
        self._rc(rc, "batch_adjoint_solve")
        return rc, [SolveInfo(i.status, i.iters, 0, i.res_norm, 0.0) for i in info]

    def upper_value_grad(self, as_, ys, xs, grads=None):
        """Batched upper-level value and gradient; returns ([g], [||grad g||])."""
        a, y, x = self._kers(as_, "a"), self._imgs(ys, "y"), self._imgs(xs, "x")
        go = self._imgs(grads, "grad_out") if grads is not None else None
        g = (ct.c_double * self.n)()
        gn = (ct.c_double * self.n)()
        self._check(L.lib().maid_batch_upper_value_grad(self.handle, a, y, x, go, g, gn, _stream()),
                    "batch_upper_value_grad")
        return list(g), list(gn)

    def hypergrad(self, thetas, as_, ys, xts, qs, with_r=True, zs=None):
        """Batched hypergradient; returns ([z], [||z||])."""
        th, y, xt, q = self._kers(thetas, "theta"), self._imgs(ys, "y"), self._imgs(xts, "x_tilde"), \
            self._imgs(qs, "q")
        a = self._kers(as_, "a") if as_ is not None else None
        if zs is None:
            zs = [torch.empty(self._kshape(i), dtype=torch.float64, device=thetas[0].device) for i in range(self.n)]
        z = self._kers(zs, "z")
        zn = (ct.c_double * self.n)()
        self._check(L.lib().maid_batch_hypergrad(self.handle, th, a, y, xt, q, int(bool(with_r)), z, zn, _stream()),
                    "batch_hypergrad")
        return zs, list(zn)

    def maid_step(self, as_, ys, states, **hp):
        """One Algorithm 2 iteration for every instance (lockstep); the states
        are updated in place.  Returns (rc, [info dict])."""
        return self.maid_steps(as_, ys, states, 0, **hp)

    def maid_steps(self, as_, ys, states, n_steps, **hp):
        """n_steps Algorithm 2 iterations for every instance in one call
        (maid_batch_steps; n_steps == 0: one maid_batch_step); an instance
        that reaches the accuracy floor or fails stops.  Returns (rc, [info
        dict]) with the counts summed over each instance's steps."""
        a, y = self._kers(as_, "a"), self._imgs(ys, "y")
        self._kers([s.theta for s in states], "theta")
        self._imgs([s.x for s in states], "x"), self._imgs([s.q for s in states], "q")
        h = dict(DEFAULT_HPARAMS)
        h.update(hp)
        hpc = L.maid_hparams(**h)
        st = (L.maid_state * self.n)(*[L.maid_state(s.theta.data_ptr(), s.x.data_ptr(), s.q.data_ptr(), s.eps,
                                                    s.delta, s.step, s.L, s.k) for s in states])
        info = (L.maid_step_info * self.n)()
        if n_steps:
            rc = L.lib().maid_batch_steps(self.handle, a, y, st, ct.byref(hpc), info, int(n_steps), _stream())
        else:
            rc = L.lib().maid_batch_step(self.handle, a, y, st, ct.byref(hpc), info, _stream())
        self._rc(rc, "batch_step")
        for s, c in zip(states, st):
            s.eps, s.delta, s.step, s.L, s.k = c.eps, c.delta, c.step, c.L, c.k
        return rc, [{f: getattr(i, f) for f, _ in L.maid_step_info._fields_} for i in info]


class Maid1D:
    """Section 4.1's 1D problem (maid1d.h): a batch of `batch` signals of n
    samples, full n x n operators, FP64.  B is (batch, n, n), A (n, n),
    vectors (batch, n), all contiguous CUDA float64 tensors."""

    def __init__(self, n, batch=1, alpha1=1.2e-3, alpha2=4e-3):
        self.n, self.batch = int(n), int(batch)
        self.alpha1, self.alpha2 = float(alpha1), float(alpha2)
        h = ct.c_void_p()
        self._h = None
        rc = L.lib().maid1d_create(ct.byref(L.maid1d_desc(self.n, self.batch, self.alpha1, self.alpha2)), ct.byref(h))
        if rc != L.OK:
            raise L.MaidError(rc, L.lib().maid1d_last_error(None).decode())
        self._h = h.value

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and L is not None and L._lib is not None:
            L._lib.maid1d_destroy(ct.c_void_p(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context is closed")
        return ct.c_void_p(self._h)

    def _t(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or \
                tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of shape {tuple(shape)}")
        return _ptr(t)

    def _vec(self, t, name):
        return self._t(t, (self.batch, self.n), name)

    def _mat(self, t, name):
        return self._t(t, (self.batch, self.n, self.n), name)

    def _per(self, v):
        v = [float(v)] * self.batch if np.isscalar(v) else [float(a) for a in v]
        if len(v) != self.batch:
            raise ValueError(f"need {self.batch} values")
        return (ct.c_double * self.batch)(*v)

    def _rc(self, rc, what):
        if rc < 0:
            raise L.MaidError(rc, f"{what}: {L.lib().maid1d_last_error(self.handle).decode()}")
        return rc

    def lower_solve(self, B, y, x, step, tol, max_iter=300):
        """maid1d_lower_solve, in place in x; returns (rc, [SolveInfo])."""
        info = (L.maid_solve_info * self.batch)()
        rc = L.lib().maid1d_lower_solve(self.handle, self._mat(B, "B"), self._vec(y, "y"), self._vec(x, "x"),
                                        float(step), self._per(tol), int(max_iter), info, _stream())
        self._rc(rc, "lower_solve")
        return rc, [SolveInfo(i.status, i.iters, 0, i.res_norm, i.L) for i in info]

    def upper_value_grad(self, A, y, x, grad=None):
        g = (ct.c_double * self.batch)()
        gn = (ct.c_double * self.batch)()
        gp = self._vec(grad, "grad") if grad is not None else None
        rc = L.lib().maid1d_upper_value_grad(self.handle, self._t(A, (self.n, self.n), "A"), self._vec(y, "y"),
                                             self._vec(x, "x"), gp, g, gn, _stream())
        self._rc(rc, "upper_value_grad")
        return list(g), list(gn)

    def adjoint_solve(self, B, x, rhs, q, tol, max_iter=1000):
        info = (L.maid_solve_info * self.batch)()
        rc = L.lib().maid1d_adjoint_solve(self.handle, self._mat(B, "B"), self._vec(x, "x"), self._vec(rhs, "rhs"),
                                          self._vec(q, "q"), self._per(tol), int(max_iter), info, _stream())
        self._rc(rc, "adjoint_solve")
        return rc, [SolveInfo(i.status, i.iters, 0, i.res_norm) for i in info]

    def hypergrad(self, B, y, x, q, z=None):
        if z is None:
            z = torch.empty((self.batch, self.n, self.n), dtype=torch.float64, device=B.device)
        zn = (ct.c_double * self.batch)()
        rc = L.lib().maid1d_hypergrad(self.handle, self._mat(B, "B"), self._vec(y, "y"), self._vec(x, "x"),
                                      self._vec(q, "q"), self._mat(z, "z"), zn, _stream())
        self._rc(rc, "hypergrad")
        return z, list(zn)

    def step(self, A, y, B, x, q, sched, lam_x=0.1, **hp):
        """maid1d_step: one Algorithm 2 iteration per instance, B, x, q in
        place; sched: list of dicts (eps, delta, step, k), updated in place.
        Returns (rc, [info dict])."""
        h = dict(DEFAULT_HPARAMS)
        h.update(hp)
        hpc = L.maid_hparams(**h)
        sc = (L.maid1d_sched * self.batch)(*[L.maid1d_sched(s["eps"], s["delta"], s["step"], s.get("k", 0))
                                             for s in sched])
        info = (L.maid_step_info * self.batch)()
        rc = L.lib().maid1d_step(self.handle, self._t(A, (self.n, self.n), "A"), self._vec(y, "y"), self._mat(B, "B"),
                                 self._vec(x, "x"), self._vec(q, "q"), sc, ct.byref(hpc), float(lam_x), info,
                                 _stream())
        self._rc(rc, "step")
        for s, c in zip(sched, sc):
            s.update(eps=c.eps, delta=c.delta, step=c.step, k=c.k)
        return rc, [{f: getattr(i, f) for f, _ in L.maid_step_info._fields_} for i in info]
