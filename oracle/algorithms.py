"""FP64 drivers of the paper's algorithms (test infrastructure only).

Each function follows the algorithm of the same name in the paper, step by
step and in its notation:

  cg        Alg. CG with CG-STEP                 (Review of Methods)
  pcg       Alg. PCG with PCG-STEP               (Review of Methods)
  cg_k      Alg. CG-K / pcg_k Alg. PCG-K          (Sections on CG-K and PCG-K)
  scg_k     Alg. S-CG-K / spcg_k Alg. S-PCG-K
  scg       Alg. S-CG with CG-PR-STEP            (Perturbation Resilient CG)
  scg_cd    Alg. S-CG-CD with CG-CD-STEP
  spcg      Alg. S-PCG with PCG-PR-STEP          (Perturbation Resilient PCG)
  perturbed the perturbation x + gamma v of eq. (superiorization) with gamma
            taken from the sequence gamma_l = gamma0 a^l (eq. gamma_sequence)

f(x) = 1/2 ||y - A x||^2 is the proximity function (the primary criterion).
The preconditioner M of the PCG family is the paper's filtered
backprojection of the residual, z = A^T F^T C F (A x - y) (Filters for
Preconditioning section); since it acts on the residual, the recursive
PCG-STEP carries the residual r = A x - y along with g = A^T r.

Readings where the paper is silent (each is stated where it is used):
  * perturbed(): v = -s/||s|| with s a TV subgradient; one global counter l
    that advances by one for every trial, accepted or not; accept when
    TV(x + gamma v) <= TV(x); at most max_trials trials, after which the point
    is left unperturbed; ||s|| = 0 leaves the point and l unchanged.
  * CG-K / PCG-K perform K steps (the text says K steps; its loop bound
    'k <= K' would give K + 1).
  * The iteration cap max_iter is not in the paper; reaching it with
    f > eps is reported as status 'noconv'.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .ops import Geometry


@dataclass
class PerturbParams:
    gamma0: float
    a: float = 0.975
    max_trials: int = 100
    kappa: float = 0.0


@dataclass
class Result:
    x: np.ndarray                 # the algorithm's output
    k: int                        # value of the counter k when the loop ended
    steps: int                    # number of (PR/CD/PCG/CG-K) steps executed
    status: str                   # 'ok' | 'noconv' | 'breakdown'
    f_out: float                  # f at the output
    trace: list = field(default_factory=list)
    records: list = field(default_factory=list)
    ell: int = 0


class Problem:
    """A, A^T, the data y and the filter, with FP64 helpers."""

    def __init__(self, geom: Geometry, y, precond_mu: Optional[float] = None):
        self.g = geom
        self.y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        assert self.y.size == geom.L
        self._kernel = None
        self.precond_mu = precond_mu

    def A(self, x):
        return self.g.project(x)

    def AT(self, r):
        return self.g.backproject(r)

    def residual(self, x):
        """A x - y."""
        return self.A(x) - self.y

    def f(self, x) -> float:
        r = self.residual(x)
        return 0.5 * float(r @ r)

    def K(self, r):
        """F^T C F applied to each projection of a sinogram-shaped vector."""
        if self._kernel is None:
            self._kernel = self.g.filter_kernel(self.precond_mu)
        return self.g.filter(r, kernel=self._kernel)

    def M_of_residual(self, r):
        """z = A^T F^T C F r, the preconditioned gradient for residual r."""
        return self.AT(self.K(r))


# ---------------------------------------------------------------------------
# Perturbation (eq. superiorization and eq. gamma_sequence)
# ---------------------------------------------------------------------------

@dataclass
class PerturbInfo:
    tv_x: float
    accepted: int        # index of the accepted trial in this call, -1 if none
    trials: int          # trials made in this call
    gamma: float         # step used (0 when the point is unperturbed)
    s_norm: float
    margins: list = field(default_factory=list)   # TV(x + gamma v) - TV(x) per trial


def perturbed(g: Geometry, x, ell: int, pp: PerturbParams):
    """Returns (x + gamma v, new l, info): v = -s/||s|| with s a subgradient of
    TV at x (a nonascending direction), gamma = gamma0 a^l for successive l
    until TV(x + gamma v) <= TV(x)."""
    s = g.tv_subgrad(x, pp.kappa)
    s_norm = float(np.sqrt(s @ s))
    tv_x = g.tv(x, pp.kappa)
    if s_norm == 0.0:
        return x.copy(), ell, PerturbInfo(tv_x, -1, 0, 0.0, 0.0)
    v = -s / s_norm
    margins = []
    for trial in range(pp.max_trials):
        gamma = pp.gamma0 * pp.a ** ell
        ell += 1
        z = x + gamma * v
        tv_z = g.tv(z, pp.kappa)
        margins.append(tv_z - tv_x)
        if tv_z <= tv_x:
            return z, ell, PerturbInfo(tv_x, trial, trial + 1, gamma, s_norm, margins)
    return x.copy(), ell, PerturbInfo(tv_x, -1, pp.max_trials, 0.0, s_norm, margins)


# ---------------------------------------------------------------------------
# CG and PCG (Review of Methods)
# ---------------------------------------------------------------------------

def cg(prob: Problem, x0, eps: float, max_iter: int = 1000) -> Result:
    """Alg. CG: k = 0, g0 = A^T(A x0 - y), p0 = -g0, delta0 = ||g0||^2; while
    f(x_k) > eps call CG-STEP; output x_k."""
    x = np.array(x0, dtype=np.float64).reshape(-1)
    g = prob.AT(prob.residual(x))
    p = -g
    delta = float(g @ g)
    k = 0
    trace = []
    fx = prob.f(x)
    status = "ok"
    while fx > eps:
        if k >= max_iter:
            status = "noconv"
            break
        # CG-STEP(A, x, p, g, delta, x', p', g', delta')
        if delta == 0.0:            # g_k = 0: x_k is a least-squares solution
            break
        h = prob.AT(prob.A(p))
        pth = float(p @ h)
        if pth == 0.0:
            status = "breakdown"
            break
        alpha = delta / pth
        x = x + alpha * p
        g = g + alpha * h
        delta_new = float(g @ g)
        beta = delta_new / delta
        p = -g + beta * p
        delta = delta_new
        k += 1
        fx = prob.f(x)
        trace.append({"k": k, "f": fx, "alpha": alpha, "beta": beta})
    return Result(x=x, k=k, steps=k, status=status, f_out=fx, trace=trace)


def _pcg_init(prob: Problem, x):
    r = prob.residual(x)
    g = prob.AT(r)
    z = prob.M_of_residual(r)
    return r, g, z


def pcg(prob: Problem, x0, eps: float, max_iter: int = 1000) -> Result:
    """Alg. PCG with PCG-STEP; z = M g is the filtered backprojection of the
    residual, so the residual is updated alongside g (r' = r + alpha A p)."""
    x = np.array(x0, dtype=np.float64).reshape(-1)
    r, g, z = _pcg_init(prob, x)
    p = -z
    delta = float(g @ z)
    k = 0
    fx = 0.5 * float(r @ r)
    status = "ok"
    trace = []
    while fx > eps:
        if k >= max_iter:
            status = "noconv"
            break
        if delta == 0.0:
            break
        q = prob.A(p)
        h = prob.AT(q)
        pth = float(p @ h)
        if pth == 0.0:
            status = "breakdown"
            break
        alpha = delta / pth
        x = x + alpha * p
        g = g + alpha * h
        r = r + alpha * q
        z = prob.M_of_residual(r)
        delta_new = float(g @ z)
        beta = delta_new / delta
        p = -z + beta * p
        delta = delta_new
        k += 1
        fx = prob.f(x)
        trace.append({"k": k, "f": fx, "alpha": alpha, "beta": beta})
    return Result(x=x, k=k, steps=k, status=status, f_out=fx, trace=trace)


def cg_k(prob: Problem, x0, K: int):
    """Alg. CG-K: K CG-STEPs from x0 with no stopping test. Returns
    (x_K, f(x0)) - f(x0) comes from the residual that forms g0."""
    x = np.array(x0, dtype=np.float64).reshape(-1)
    r = prob.residual(x)
    f0 = 0.5 * float(r @ r)
    g = prob.AT(r)
    p = -g
    delta = float(g @ g)
    for _ in range(K):
        if delta == 0.0:
            break
        h = prob.AT(prob.A(p))
        pth = float(p @ h)
        if pth == 0.0:
            break
        alpha = delta / pth
        x = x + alpha * p
        g = g + alpha * h
        delta_new = float(g @ g)
        beta = delta_new / delta
        p = -g + beta * p
        delta = delta_new
    return x, f0


def pcg_k(prob: Problem, x0, K: int):
    """Alg. PCG-K: K PCG-STEPs from x0. Returns (x_K, f(x0))."""
    x = np.array(x0, dtype=np.float64).reshape(-1)
    r, g, z = _pcg_init(prob, x)
    f0 = 0.5 * float(r @ r)
    p = -z
    delta = float(g @ z)
    for _ in range(K):
        if delta == 0.0:
            break
        q = prob.A(p)
        h = prob.AT(q)
        pth = float(p @ h)
        if pth == 0.0:
            break
        alpha = delta / pth
        x = x + alpha * p
        g = g + alpha * h
        r = r + alpha * q
        z = prob.M_of_residual(r)
        delta_new = float(g @ z)
        beta = delta_new / delta
        p = -z + beta * p
        delta = delta_new
    return x, f0


def _s_k(prob: Problem, x0, eps, pp: PerturbParams, K: int, inner, max_iter: int,
         record: bool = False) -> Result:
    """Alg. S-CG-K / S-PCG-K: k = 0, x_{-1/2} = x0; while f(x_{k-1/2}) > eps:
    x_{k+1/2} = perturbed(x_k), x_{k+1} = inner-K(x_{k+1/2}), k = k + 1;
    output x_{k-1/2}."""
    x = np.array(x0, dtype=np.float64).reshape(-1)
    x_half = x.copy()
    f_half = prob.f(x_half)
    k, ell = 0, 0
    status = "ok"
    trace, records = [], []
    while f_half > eps:
        if k >= max_iter:
            status = "noconv"
            break
        x_half, ell, info = perturbed(prob.g, x, ell, pp)
        x, f_half = inner(prob, x_half, K)
        k += 1
        trace.append({"k": k, "f_half": f_half, "tv_x": info.tv_x, "accepted": info.accepted,
                      "trials": info.trials, "ell": ell, "gamma": info.gamma,
                      "margins": info.margins})
        if record:
            records.append({"k": k, "x_half": x_half})
    return Result(x=x_half, k=k, steps=k, status=status, f_out=f_half, trace=trace,
                  records=records, ell=ell)


def scg_k(prob: Problem, x0, eps: float, pp: PerturbParams, K: int = 2,
          max_iter: int = 1000, record: bool = False) -> Result:
    return _s_k(prob, x0, eps, pp, K, cg_k, max_iter, record)


def spcg_k(prob: Problem, x0, eps: float, pp: PerturbParams, K: int = 2,
           max_iter: int = 1000) -> Result:
    return _s_k(prob, x0, eps, pp, K, pcg_k, max_iter)


# ---------------------------------------------------------------------------
# Perturbation-resilient variants
# ---------------------------------------------------------------------------

PerturbFn = Callable[[np.ndarray, int, dict], np.ndarray]


def scg(prob: Problem, x0, eps: float, pp: PerturbParams, max_iter: int = 1000,
        perturb_fn: Optional[PerturbFn] = None, record: bool = False) -> Result:
    """Alg. S-CG with CG-PR-STEP.

    perturb_fn(x_k, k, ctx) -> x_{k+1/2} replaces perturbed() when given
    (used by tests that force perturbations of a prescribed size)."""
    x0 = np.array(x0, dtype=np.float64).reshape(-1)
    # Steps 1-7 of S-CG.
    x_half = x0.copy()                          # x_{1/2} = x0
    r = prob.residual(x0)
    f_half = 0.5 * float(r @ r)                 # f(x_{1/2})
    g = prob.AT(r)                              # g0
    p = -g                                      # p0
    q = prob.A(p)
    h = prob.AT(q)                              # h0 = A^T A p0
    pth = float(p @ h)
    if pth == 0.0:
        return Result(x=x_half, k=1, steps=0, status="breakdown", f_out=f_half)
    alpha = -float(g @ p) / pth
    x = x0 + alpha * p                          # x1
    k, ell = 1, 0
    trace, records = [], []
    status = "ok"
    while f_half > eps:                         # f(x_{k-1/2}) > eps
        if k - 1 >= max_iter:
            status = "noconv"
            break
        if perturb_fn is None:
            xh, ell, info = perturbed(prob.g, x, ell, pp)
        else:
            xh = perturb_fn(x, k, {"prob": prob})
            info = PerturbInfo(float("nan"), -1, 0, 0.0, 0.0)
        # CG-PR-STEP(A, y, x_{k+1/2}, p_{k-1}, h_{k-1}, x_{k+1}, p_k, h_k)
        r = prob.residual(xh)
        f_half = 0.5 * float(r @ r)             # f(x_{k+1/2})
        g_new = prob.AT(r)                      # g' = A^T(A x - y)
        beta = float(g_new @ h) / pth           # beta = g'^T h / p^T h
        p_new = -g_new + beta * p               # p' = -g' + beta p
        q_new = prob.A(p_new)
        h_new = prob.AT(q_new)                  # h' = A^T A p'
        pth_new = float(p_new @ h_new)
        if pth_new == 0.0:
            status = "breakdown"
            x_half = xh
            k += 1
            break
        gp = float(g_new @ p_new)
        alpha = -gp / pth_new                   # alpha = -g'^T p' / p'^T h'
        x_new = xh + alpha * p_new              # x' = x + alpha p'
        trace.append({"k": k, "f_half": f_half, "tv_x": info.tv_x, "accepted": info.accepted,
                      "trials": info.trials, "ell": ell, "gamma": info.gamma,
                      "margins": info.margins, "beta": beta, "alpha": alpha, "gp": gp,
                      "qq": pth_new})
        if record:
            records.append({"k": k, "x_k": x, "x_half": xh, "g_half": g_new, "p_prev": p,
                            "q_prev": q, "p": p_new, "q": q_new, "x_next": x_new,
                            "f_half": f_half})
        x_half, x, p, h, q, pth = xh, x_new, p_new, h_new, q_new, pth_new
        k += 1
    return Result(x=x_half, k=k, steps=len(trace), status=status, f_out=f_half, trace=trace,
                  records=records, ell=ell)


def scg_3op(prob: Problem, x0, eps: float, pp: PerturbParams, max_iter: int = 1000) -> Result:
    """Alg. S-CG with CG-PR-STEP rewritten with q = A p carried by linearity.

    With h = A^T A p: p^T h = ||A p||^2 and g'^T h = (A g')^T (A p), so beta =
    (A g')^T q / ||q||^2; and A p' = A(-g' + beta p) = -A g' + beta q. A step
    then needs A x_{k+1/2}, A^T r and A g' (two projections and one
    backprojection) instead of two of each. The same iteration in exact
    arithmetic; q accumulates rounding like a recursive residual."""
    x0 = np.array(x0, dtype=np.float64).reshape(-1)
    x_half = x0.copy()
    r = prob.residual(x0)
    f_half = 0.5 * float(r @ r)
    g = prob.AT(r)
    p = -g
    q = prob.A(p)                               # q0 = A p0
    qq = float(q @ q)
    if qq == 0.0:
        return Result(x=x_half, k=1, steps=0, status="breakdown", f_out=f_half)
    alpha = -float(g @ p) / qq
    x = x0 + alpha * p
    k, ell = 1, 0
    trace = []
    status = "ok"
    while f_half > eps:
        if k - 1 >= max_iter:
            status = "noconv"
            break
        xh, ell, info = perturbed(prob.g, x, ell, pp)
        r = prob.residual(xh)
        f_half = 0.5 * float(r @ r)
        g_new = prob.AT(r)
        u = prob.A(g_new)                       # A g'
        beta = float(u @ q) / qq                # (A g')^T q / ||q||^2
        p_new = -g_new + beta * p
        q_new = -u + beta * q                   # A p' by linearity
        qq_new = float(q_new @ q_new)
        if qq_new == 0.0:
            status = "breakdown"
            x_half = xh
            k += 1
            break
        gp = float(g_new @ p_new)
        alpha = -gp / qq_new
        x_new = xh + alpha * p_new
        trace.append({"k": k, "f_half": f_half, "tv_x": info.tv_x, "accepted": info.accepted,
                      "trials": info.trials, "ell": ell, "gamma": info.gamma,
                      "margins": info.margins, "beta": beta, "alpha": alpha, "gp": gp,
                      "qq": qq_new})
        x_half, x, p, q, qq = xh, x_new, p_new, q_new, qq_new
        k += 1
    return Result(x=x_half, k=k, steps=len(trace), status=status, f_out=f_half, trace=trace,
                  ell=ell)


def scg_cd(prob: Problem, x0, eps: float, pp: PerturbParams, max_iter: int = 1000,
           record: bool = False) -> Result:
    """Alg. S-CG-CD with CG-CD-STEP (beta = -||g'||^2 / g^T p, the
    conjugate-descent rule); the step carries g instead of h."""
    x0 = np.array(x0, dtype=np.float64).reshape(-1)
    x_half = x0.copy()
    r = prob.residual(x0)
    f_half = 0.5 * float(r @ r)
    g = prob.AT(r)
    p = -g
    h = prob.AT(prob.A(p))
    pth = float(p @ h)
    if pth == 0.0:
        return Result(x=x_half, k=1, steps=0, status="breakdown", f_out=f_half)
    alpha = -float(g @ p) / pth
    x = x0 + alpha * p
    k, ell = 1, 0
    trace, records = [], []
    status = "ok"
    while f_half > eps:
        if k - 1 >= max_iter:
            status = "noconv"
            break
        xh, ell, info = perturbed(prob.g, x, ell, pp)
        # CG-CD-STEP(A, y, x_{k+1/2}, p_{k-1}, g_{k-1}, x_{k+1}, p_k, g_k)
        r = prob.residual(xh)
        f_half = 0.5 * float(r @ r)
        g_new = prob.AT(r)
        beta = -float(g_new @ g_new) / float(g @ p)
        p_new = -g_new + beta * p
        h_new = prob.AT(prob.A(p_new))
        pth_new = float(p_new @ h_new)
        if pth_new == 0.0:
            status = "breakdown"
            x_half = xh
            k += 1
            break
        gp = float(g_new @ p_new)
        alpha = -gp / pth_new
        x_new = xh + alpha * p_new
        trace.append({"k": k, "f_half": f_half, "tv_x": info.tv_x, "accepted": info.accepted,
                      "trials": info.trials, "ell": ell, "gamma": info.gamma,
                      "margins": info.margins, "beta": beta, "alpha": alpha, "gp": gp,
                      "qq": pth_new})
        if record:
            records.append({"k": k, "x_k": x, "x_half": xh, "p": p_new, "x_next": x_new})
        x_half, x, p, g = xh, x_new, p_new, g_new
        k += 1
    return Result(x=x_half, k=k, steps=len(trace), status=status, f_out=f_half, trace=trace,
                  records=records, ell=ell)


def spcg(prob: Problem, x0, eps: float, pp: PerturbParams, max_iter: int = 1000) -> Result:
    """Alg. S-PCG with PCG-PR-STEP: z' = M g' (filtered backprojection of the
    residual), beta = z'^T h / p^T h, p' = -z' + beta p."""
    x0 = np.array(x0, dtype=np.float64).reshape(-1)
    x_half = x0.copy()
    r = prob.residual(x0)
    f_half = 0.5 * float(r @ r)
    g = prob.AT(r)                              # g0
    z = prob.M_of_residual(r)                   # z0 = M g0
    p = -z                                      # p0 = -z0
    h = prob.AT(prob.A(p))                      # h0
    pth = float(p @ h)
    if pth == 0.0:
        return Result(x=x_half, k=1, steps=0, status="breakdown", f_out=f_half)
    alpha = -float(g @ p) / pth
    x = x0 + alpha * p
    k, ell = 1, 0
    trace = []
    status = "ok"
    while f_half > eps:
        if k - 1 >= max_iter:
            status = "noconv"
            break
        xh, ell, info = perturbed(prob.g, x, ell, pp)
        # PCG-PR-STEP(A, y, x_{k+1/2}, p_{k-1}, h_{k-1}, x_{k+1}, p_k, h_k, M)
        r = prob.residual(xh)
        f_half = 0.5 * float(r @ r)
        g_new = prob.AT(r)                      # g'
        z_new = prob.M_of_residual(r)           # z' = M g'
        beta = float(z_new @ h) / pth           # beta = z'^T h / p^T h
        p_new = -z_new + beta * p               # p' = -z' + beta p
        h_new = prob.AT(prob.A(p_new))          # h' = A^T A p'
        pth_new = float(p_new @ h_new)
        if pth_new == 0.0:
            status = "breakdown"
            x_half = xh
            k += 1
            break
        gp = float(g_new @ p_new)
        alpha = -gp / pth_new                   # alpha = -g'^T p' / p'^T h'
        x_new = xh + alpha * p_new
        trace.append({"k": k, "f_half": f_half, "tv_x": info.tv_x, "accepted": info.accepted,
                      "trials": info.trials, "ell": ell, "gamma": info.gamma,
                      "margins": info.margins, "beta": beta, "alpha": alpha, "gp": gp,
                      "qq": pth_new})
        x_half, x, p, h, pth = xh, x_new, p_new, h_new, pth_new
        k += 1
    return Result(x=x_half, k=k, steps=len(trace), status=status, f_out=f_half, trace=trace,
                  ell=ell)


def power_norm2(prob: Problem, iters: int = 200, seed: int = 0) -> float:
    """c^2 = ||A^T A||_2 (the paper's c is ||A||_2, eq. lambda) by power
    iteration on A^T A."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(prob.g.J)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = prob.AT(prob.A(v))
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def ls_floor_dense(geom: Geometry, y) -> tuple[float, np.ndarray]:
    """eps0 = min_x 1/2 ||y - A x||^2 (eq. epsilon_0) by a dense least-squares
    solve; returns (eps0, minimum-norm x_LS). Tiny problems only."""
    A = geom.dense()
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    x, *_ = np.linalg.lstsq(A, y, rcond=None)
    r = A @ x - y
    return 0.5 * float(r @ r), x


def ls_floor_cg(prob: Problem, tol: float = 1e-10, max_iter: int = 5000) -> float:
    """Upper bound of eps0 from plain CG run until ||g_k|| <= tol ||g_0||."""
    x = np.zeros(prob.g.J)
    g = prob.AT(prob.residual(x))
    p = -g
    delta = float(g @ g)
    g0 = np.sqrt(delta)
    for _ in range(max_iter):
        if np.sqrt(delta) <= tol * g0:
            break
        h = prob.AT(prob.A(p))
        alpha = delta / float(p @ h)
        x = x + alpha * p
        g = g + alpha * h
        delta_new = float(g @ g)
        p = -g + (delta_new / delta) * p
        delta = delta_new
    return prob.f(x)
