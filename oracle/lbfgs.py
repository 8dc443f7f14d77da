"""Preconditioned L-BFGS with the Hager-Zhang line search: the plain oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper optimises the iPEPS energy with L-BFGS (history m = 200, Hager-Zhang
line search, Sec. IV A) into which the preconditioned gradient P^-1 g of
Sec. II (Eqs. (1)-(4)) enters as the initial inverse-Hessian approximation,
with the regularised local metric P = N_local + delta I of Sec. III B and an
adaptive delta = |E_{i+1} - E_i| or |g|^2 (Sec. III B).  Written here from the
standard descriptions (Nocedal & Wright, Numerical Optimization, the two-loop
recursion; Hager & Zhang, SIAM J. Optim. 16 (2005) 170, the line search with
its bracket / update / secant^2 steps and the Wolfe and approximate Wolfe
conditions), in plain float64 numpy on flat parameter vectors.

Readings where the paper is silent (the same in the device optimiser):
  * two-loop recursion with H_0 = P^-1 (one preconditioner solve per
    iteration, at the current point, no further scaling); without the
    preconditioner H_0 = gamma I, gamma = s^T y / y^T y of the newest pair
    (1 before the first pair);
  * first trial step c = 1 with the preconditioner, c = psi0 max|x| / max|g|
    (psi0 = 0.01) for the first iteration without it, c = 1 afterwards;
  * a pair (s, y) enters the history only when s^T y > 1e-12 |s| |y|; the
    oldest of m pairs is dropped;
  * the line search accepts the first evaluated step that meets the Wolfe
    (T1) or the approximate Wolfe (T2) condition of Hager and Zhang with
    delta = 0.1, sigma = 0.9, eps = 1e-6 |f(x_k)|, theta = 0.5, gamma =
    0.66, rho = 5; after max_evals evaluations it takes the evaluated step
    with the lowest energy (and re-evaluates there);
  * delta of the next iteration: mode "energy" |E_{k+1} - E_k|, mode
    "gradient" |g_{k+1}|^2, mode "fixed" delta0; clamped to
    [delta_min, delta_max].

Parity status: the line search is pinned on closed-form one-dimensional
functions and the whole optimiser on quadratics, where preconditioning with
the exact Hessian reaches the minimiser in one step (Eq. (5)), and on a
Rosenbrock valley (tests/test_oracle_lbfgs.py).
"""
from __future__ import annotations

import numpy as np

HZ = dict(delta=0.1, sigma=0.9, eps=1e-6, theta=0.5, gamma=0.66, rho=5.0)


class LineSearchFailed(RuntimeError):
    pass


def hager_zhang(phi, c, phi0, dphi0, fscale, max_evals=20, p=HZ):
    """Step length along a descent direction.

    phi(a) -> (phi(a), phi'(a)); phi0 = phi(0), dphi0 = phi'(0) < 0;
    fscale = |f(x_k)| (the approximate-Wolfe slack is eps * fscale).
    Returns (a, phi(a), phi'(a), evaluations, ok); ok is False when no step
    met the conditions within max_evals (then a is the evaluated step with
    the lowest phi, and its values)."""
    if not dphi0 < 0:
        raise LineSearchFailed("not a descent direction")
    eps_k = p["eps"] * fscale
    thresh = phi0 + eps_k
    seen = {}           # a -> (phi, dphi)
    order = []

    class Done(Exception):
        pass

    def ev(a):
        if a in seen:
            return seen[a]
        if len(order) >= max_evals:
            raise Done()
        v = phi(a)
        seen[a] = v
        order.append(a)
        f, df = v
        wolfe = (p["delta"] * dphi0 * a >= f - phi0) and (df >= p["sigma"] * dphi0)
        approx = ((2 * p["delta"] - 1) * dphi0 >= df >= p["sigma"] * dphi0
                  and f <= thresh)
        if wolfe or approx:
            raise Found(a)
        return v

    class Found(Exception):
        def __init__(self, a):
            self.a = a

    def bisect_update(a, b):
        # U3: phi'(b) < 0 and phi(b) > thresh: shrink [a, b] by theta steps
        while True:
            d = (1 - p["theta"]) * a + p["theta"] * b
            f, df = ev(d)
            if df >= 0:
                return a, d
            if f <= thresh:
                a = d
            else:
                b = d

    def update(a, b, c):
        if not (a < c < b):
            return a, b
        f, df = ev(c)
        if df >= 0:
            return a, c
        if f <= thresh:
            return c, b
        return bisect_update(a, c)

    def secant(a, b):
        da, db = seen[a][1] if a in seen else dphi0, seen[b][1]
        if db == da:
            return 0.5 * (a + b)
        return (a * db - b * da) / (db - da)

    def secant2(a, b):
        c = secant(a, b)
        A, B = update(a, b, c)
        if c == B:
            cb = secant(b, B)
            return update(A, B, cb)
        if c == A:
            cb = secant(a, A)
            return update(A, B, cb)
        return A, B

    def bracket(c):
        cs = []
        while True:
            f, df = ev(c)
            cs.append((c, f))
            if df >= 0:
                a = 0.0
                for ci, fi in cs[:-1]:
                    if fi <= thresh:
                        a = ci
                return a, c
            if f > thresh:
                return bisect_update(0.0, c)
            c = p["rho"] * c

    try:
        a, b = bracket(c)
        while True:
            A, B = secant2(a, b)
            if B - A > p["gamma"] * (b - a):
                A, B = update(A, B, 0.5 * (A + B))
            if (A, B) == (a, b):
                # no progress possible in floating point
                raise Done()
            a, b = A, B
    except Found as fd:
        f, df = seen[fd.a]
        return fd.a, f, df, len(order), True
    except Done:
        best = min(order, key=lambda t: seen[t][0]) if order else 0.0
        if not order:
            return 0.0, phi0, dphi0, 0, False
        f, df = seen[best]
        return best, f, df, len(order), False


def two_loop(g, S, Y, apply_h0):
    """r = H g by the two-loop recursion over the pairs (oldest first in S,
    Y) with the initial inverse Hessian apply_h0(q)."""
    q = g.copy()
    k = len(S)
    rho = [1.0 / float(Y[i] @ S[i]) for i in range(k)]
    alpha = [0.0] * k
    for i in range(k - 1, -1, -1):
        alpha[i] = rho[i] * float(S[i] @ q)
        q = q - alpha[i] * Y[i]
    r = apply_h0(q)
    for i in range(k):
        beta = rho[i] * float(Y[i] @ r)
        r = r + S[i] * (alpha[i] - beta)
    return r


def minimize(fg, x0, n_iter, precond=None, m=200, delta_mode="energy",
             delta0=1e-2, delta_min=1e-12, delta_max=1.0, max_evals=20,
             psi0=0.01, hz=HZ):
    """L-BFGS on f with gradient, optionally preconditioned.

    fg(x) -> (f, g) evaluates at x (the iPEPS problem converges its
    environment there); precond(x, g, delta) -> P(x)^-1 g at the point of
    the LAST fg call, which is always x.  Returns a list of per-iteration
    records (x, f, g, alpha, evaluations, delta, line-search ok)."""
    x = np.array(x0, dtype=np.float64).ravel()
    f, g = fg(x)
    g = np.asarray(g, dtype=np.float64).ravel()
    S, Y = [], []
    delta = delta0
    hist = [dict(x=x.copy(), f=f, g=g.copy(), alpha=0.0, evals=1,
                 delta=delta, ok=True)]
    for it in range(n_iter):
        if precond is not None:
            h0 = lambda q: np.asarray(precond(x, q, delta),  # noqa: E731
                                      dtype=np.float64).ravel()
        else:
            gam = (float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])) if S else 1.0
            h0 = lambda q: gam * q  # noqa: E731
        d = -two_loop(g, S, Y, h0)
        dphi0 = float(g @ d)
        if not dphi0 < 0:
            # lost descent (curvature pairs inconsistent): restart
            S, Y = [], []
            d = -h0(g)
            dphi0 = float(g @ d)
            if not dphi0 < 0:
                break   # stationary point: no descent direction left
        if it == 0 and precond is None:
            c = psi0 * np.abs(x).max() / np.abs(g).max()
        else:
            c = 1.0
        cache = {}

        def phi(a):
            fa, ga = fg(x + a * d)
            ga = np.asarray(ga, dtype=np.float64).ravel()
            cache[a] = (fa, ga)
            dfa = float(ga @ d)
            if not (np.isfinite(fa) and np.isfinite(dfa)):
                return np.inf, np.inf    # unusable point: move back
            return fa, dfa

        a, fa, dfa, nev, ok = hager_zhang(phi, c, f, dphi0, abs(f),
                                         max_evals, hz)
        if not np.isfinite(fa):
            a = 0.0                      # no usable point: stay at x
        if a in cache:
            fa, ga = cache[a]
        if not ok or order_last(cache) != a:
            # make the accepted point the last evaluated one
            fa, ga = fg(x + a * d)
            ga = np.asarray(ga, dtype=np.float64).ravel()
            nev += 1
        s = a * d
        y = ga - g
        if float(s @ y) > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        if delta_mode == "energy":
            delta = abs(fa - f)
        elif delta_mode == "gradient":
            delta = float(ga @ ga)
        else:
            delta = delta0
        delta = min(max(delta, delta_min), delta_max)
        x = x + s
        f, g = fa, ga
        hist.append(dict(x=x.copy(), f=f, g=g.copy(), alpha=a, evals=nev,
                         delta=delta, ok=ok))
    return hist


def order_last(cache):
    """The most recently inserted key of a dict."""
    return next(reversed(cache)) if cache else None


class IpepsProblem:
    """Energy, gradient and preconditioner of an iPEPS for minimize().

    Every evaluation converges the environment from the previous
    evaluation's (the trace boundary for the first) to ctm_tol, then takes
    the K-step gradient (Sec. IV A); the preconditioner is the local metric
    of that environment (Eq. (11)) solved by CG (Sec. III C)."""

    def __init__(self, shape, terms, chi, ctm_tol=1e-10, ctm_max_iter=200,
                 K=20, cg_tol=0.0, cg_maxiter=20, gmres_m=30,
                 fd_step=1e-5):
        self.shape, self.terms, self.chi = tuple(shape), terms, chi
        self.ctm_tol, self.ctm_max_iter, self.K = ctm_tol, ctm_max_iter, K
        self.cg_tol, self.cg_maxiter = cg_tol, cg_maxiter
        self.gmres_m, self.fd_step = gmres_m, fd_step
        self.env = None
        self.evals = 0

    def fg(self, x):
        from . import ctmrg, gradient
        A = np.asarray(x).reshape(self.shape)
        self.env, _, _ = ctmrg.converge(A, self.chi, self.ctm_tol,
                                        self.ctm_max_iter, env=self.env)
        e, g = gradient.grad_K(A, self.terms, self.env, self.chi, self.K)
        self.evals += 1
        return float(e), g.numpy().ravel()

    def precond_bp(self, x, g, delta):
        """The belief-propagation (chi = 1) metric at x (Sec. III A)."""
        from . import bp
        A = np.asarray(x).reshape(self.shape)
        xg, _, _ = bp.precondition_bp(A, np.asarray(g).reshape(self.shape),
                                      delta, self.ctm_tol, self.ctm_max_iter)
        return xg.numpy().ravel()

    def precond(self, x, g, delta):
        from . import metric
        A = np.asarray(x).reshape(self.shape)
        xg, _, _, _ = metric.precondition(
            self.env, A, np.asarray(g).reshape(self.shape), delta,
            self.cg_tol, self.cg_maxiter)
        return xg.numpy().ravel()

    def precond_local_gmres(self, x, g, delta):
        """The local metric solved by one GMRES cycle (Sec. III C)."""
        from . import full_metric
        A = np.asarray(x).reshape(self.shape)
        xg, _, _ = full_metric.precondition_local_gmres(
            self.env, A, np.asarray(g).reshape(self.shape), delta,
            self.gmres_m, self.cg_tol)
        return xg.numpy().ravel()

    def precond_full(self, x, g, delta):
        """The full metric (Eq. (10)) solved by one GMRES cycle, 1x1 cell."""
        from . import full_metric
        A = np.asarray(x).reshape(self.shape)
        xg, _, _ = full_metric.precondition_full(
            A, np.asarray(g).reshape(self.shape), self.env, self.chi, self.K,
            delta, self.gmres_m, self.cg_tol, self.fd_step)
        return np.asarray(xg).ravel()
