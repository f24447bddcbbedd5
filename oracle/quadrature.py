"""Oracle: minimax Laplace quadrature for the energy denominator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

The paper replaces 1/D (D = e_i + e_j - e_a - e_b < 0) by a Laplace
integral evaluated with a few tau points (Eq. SCHLT and the LTMP2
subsection; the quadrature itself is only cited, Haser 1992 / Kaltak 2014).
The reading used here is the relative-error minimax exponential sum

    1/x  ~  sum_n w_n exp(-x tau_n),   x in [x_min, x_max],

computed by the Remez exchange for exponential sums (Takatsuka, Ten-no and
Hackbusch, J. Chem. Phys. 129, 044112 (2008); theory: Braess and Hackbusch).
Work in y = x / x_min in [1, R], R = x_max / x_min, with
s(y) = sum_n beta_n exp(-alpha_n y), alpha = exp(p), beta = exp(q), and the
error curve e(y) = y s(y) - 1.  The best approximation equioscillates at
2N + 1 points (alternation theorem for this varisolvent family).

Steps (all FP64, plain numpy):
  1. start at R_s(N) = max(10, exp(1.25 (N - 1) - 2)), where the error is
     ~1e-3 and a uniform bump layout is in the right basin: exponents from
     a uniform grid of s = -log(alpha) on [-1, log R_s + 1], weights of the
     trapezoid rule of 1/x = int exp(-x e^s + s) ds, refined by
     Levenberg-Marquardt least squares and Lawson reweighting;
  2. Remez exchange: locate the 2N + 1 alternating extrema of e (dense log
     grid, then Newton on de/dt = 0), Newton-solve e(y_k) = (-1)^k E for
     (p, q, E), repeat until the extrema levels agree to 1e-8 relative;
  3. continuation in R from R_s to the target with adaptive steps, each
     step seeded with the previous reference stretched in log y;
  4. tau_n = alpha_n / x_min, w_n = beta_n / x_min (sorted ascending in tau).
"""

from __future__ import annotations

import math

import numpy as np

__all__ = ["minimax_laplace", "minimax_unit", "r_floor", "rel_error_curve", "max_rel_error",
           "alternation_points"]


def _err(y, p, q):
    a = np.exp(p)
    b = np.exp(q)
    return y * (np.exp(-np.outer(y, a)) @ b) - 1.0


def _jac(y, p, q):
    a = np.exp(p)
    b = np.exp(q)
    E = np.exp(-np.outer(y, a)) * b[None, :]
    dq = y[:, None] * E
    dp = -(y[:, None] ** 2) * a[None, :] * E
    return np.concatenate([dp, dq], axis=1)


def _dt_derivs(t, p, q):
    """d e / dt and d^2 e / dt^2 with y = exp(t)."""
    y = np.exp(t)
    a = np.exp(p)
    b = np.exp(q)
    E = np.exp(-np.outer(y, a)) * b[None, :]
    s0 = E.sum(1)
    s1 = -(E * a[None, :]).sum(1)
    s2 = (E * (a * a)[None, :]).sum(1)
    g1 = s0 + y * s1                 # d(y s)/dy
    g2 = 2.0 * s1 + y * s2           # d^2(y s)/dy^2
    return y * g1, y * g1 + y * y * g2


def alternation_points(N, R, p, q, ngrid=20000):
    """Alternating extrema of e on [1, R]: endpoints plus interior extrema.

    Interior extrema are bracketed on a uniform grid in t = log y and refined
    by Newton on de/dt = 0.  Neighbours of equal sign are merged (the larger
    |e| kept); surplus points are dropped from the end with smaller |e|.
    """
    T = math.log(R)
    t = np.linspace(0.0, T, ngrid)
    e = _err(np.exp(t), p, q)
    de = np.diff(e)
    k = np.nonzero(de[:-1] * de[1:] < 0)[0] + 1
    tk = t[k].copy()
    h = t[1] - t[0]
    for _ in range(30):
        d1, d2 = _dt_derivs(tk, p, q)
        ok = d2 != 0
        step = np.zeros_like(tk)
        step[ok] = -d1[ok] / d2[ok]
        step = np.clip(step, -h, h)
        tk = tk + step
        if np.abs(step).max(initial=0.0) < 1e-15 * max(1.0, T):
            break
    tk = np.clip(tk, 0.0, T)
    ts = np.concatenate([[0.0], tk, [T]])
    ys = np.exp(ts)
    es = _err(ys, p, q)
    sel_y, sel_e = [ys[0]], [es[0]]
    for yy, ee in zip(ys[1:], es[1:]):
        if np.sign(ee) == np.sign(sel_e[-1]):
            if abs(ee) > abs(sel_e[-1]):
                sel_y[-1], sel_e[-1] = yy, ee
        else:
            sel_y.append(yy)
            sel_e.append(ee)
    while len(sel_y) > 2 * N + 1:
        if abs(sel_e[0]) < abs(sel_e[-1]):
            sel_y.pop(0)
            sel_e.pop(0)
        else:
            sel_y.pop()
            sel_e.pop()
    return np.array(sel_y), np.array(sel_e), float(np.abs(e).max())


def _newton_reference(N, ys, p, q, E, maxit=40):
    """Solve e(y_k) = (-1)^k E (k = 0..2N) for (p, q, E); damped Newton."""
    alt = np.array([(-1.0) ** k for k in range(2 * N + 1)])
    x = np.concatenate([p, q, [E]])
    F = _err(ys, x[:N], x[N:2 * N]) - alt * x[-1]
    for _ in range(maxit):
        J = np.concatenate([_jac(ys, x[:N], x[N:2 * N]), -alt[:, None]], axis=1)
        try:
            step = np.linalg.solve(J, -F)
        except np.linalg.LinAlgError:
            return None
        lam = 1.0
        f0 = np.abs(F).max()
        while True:
            xn = x + lam * step
            with np.errstate(all="ignore"):
                Fn = _err(ys, xn[:N], xn[N:2 * N]) - alt * xn[-1]
            if np.all(np.isfinite(Fn)) and np.abs(Fn).max() <= f0:
                break
            lam *= 0.5
            if lam < 1e-8:
                # no descent left: accept if already at the evaluation noise
                return x if f0 <= 1e-3 * abs(x[-1]) else None
        x, F = xn, Fn
        if np.abs(F).max() <= max(1e-13 * abs(x[-1]), 2e-16):
            break
    return x


def _remez(N, R, p, q, ref=None, tol=1e-8, maxit=60):
    """Remez exchange from (p, q); returns (p, q, delta, reference) or None."""
    if ref is not None:
        e0 = _err(ref, p, q)
        x = _newton_reference(N, ref, p, q, np.abs(e0).mean() * np.sign(e0[0]))
        if x is None:
            return None
        p, q = x[:N], x[N:2 * N]
    for _ in range(maxit):
        ys, es, emax = alternation_points(N, R, p, q)
        if len(ys) < 2 * N + 1:
            return None
        lo = np.abs(es).min()
        spread = (np.abs(es).max() - lo) / lo
        if spread <= max(tol, 4e-15 / lo):
            return p, q, emax, ys
        x = _newton_reference(N, ys, p, q, np.abs(es).mean() * np.sign(es[0]))
        if x is None:
            return None
        p, q = x[:N], x[N:2 * N]
        o = np.argsort(p)
        p, q = p[o], q[o]
    return None


def _lm(N, y, p, q, w, iters):
    """Levenberg-Marquardt on sum_k (w_k e(y_k))^2 over (p, q)."""
    x = np.concatenate([p, q])
    lam = 1e-2
    r = _err(y, x[:N], x[N:]) * w
    f = r @ r
    for _ in range(iters):
        J = _jac(y, x[:N], x[N:]) * w[:, None]
        A = J.T @ J
        g = J.T @ r
        D = np.diag(np.maximum(np.diag(A), 1e-30))
        moved = False
        for _ in range(60):
            step = np.linalg.lstsq(A + lam * D, -g, rcond=None)[0]
            xn = x + step
            with np.errstate(all="ignore"):
                rn = _err(y, xn[:N], xn[N:]) * w
                fn = rn @ rn
            if np.isfinite(fn) and fn < f:
                moved = True
                break
            lam *= 3.0
        if not moved:
            break
        gain = (f - fn) / f
        x, r, f = xn, rn, fn
        lam = max(lam / 3.0, 1e-15)
        if gain < 1e-14:
            break
    return x[:N], x[N:]


def _start(N):
    """Minimax fit at the well-conditioned start R_s(N) (step 1 + 2)."""
    Rs = max(10.0, math.exp(1.25 * (N - 1) - 2.0))
    T = math.log(Rs)
    if N == 1:
        p = np.array([-T / 2.0])
        q = p + 1.4
    else:
        s = np.linspace(-1.0, T + 1.0, N)
        p = -s
        q = -s + math.log(s[1] - s[0])
        y = np.exp(np.linspace(0.0, T, 3000))
        w = np.ones_like(y)
        p, q = _lm(N, y, p, q, w, 500)
        for _ in range(30):
            e = np.abs(_err(y, p, q))
            w = w * (e / e.max()) ** 0.5 + 1e-300
            w /= w.max()
            p, q = _lm(N, y, p, q, np.sqrt(w), 100)
    res = _remez(N, Rs, p, q)
    if res is None:
        raise RuntimeError(f"minimax start failed for N={N}")
    return Rs, res


def _walk(N, R0, res, R):
    """Continuation in R with adaptive log-steps (step 3)."""
    p, q, d, ys = res
    cur = R0
    lf = 0.25
    n_steps = 0
    while abs(math.log(cur / R)) > 1e-13:
        dl = math.log(R / cur)
        nxt = cur * math.exp(max(-lf, min(lf, dl)))
        if abs(math.log(nxt / R)) < 1e-13:
            nxt = R
        ref = np.exp(np.log(ys) * math.log(nxt) / math.log(cur))
        out = _remez(N, nxt, p, q, ref=ref)
        n_steps += 1
        if n_steps > 2000:
            raise RuntimeError("minimax continuation did not reach the target")
        if out is not None:
            p, q, d, ys = out
            cur = nxt
            lf = min(0.4, lf * 1.5)
        else:
            lf *= 0.5
            if lf < 1e-4:
                raise RuntimeError(f"minimax continuation stalled at R={cur:g} (N={N})")
    return p, q, d, ys


_START_CACHE: dict = {}


def r_floor(N: int) -> float:
    """Smallest R at which the N-term fit is computed (FP64 floor).

    Below it the minimax error falls under ~1e-8, where the Remez Newton
    system is no longer solvable in double precision.  A request with
    R < r_floor(N) gets the fit for [1, r_floor(N)], which contains [1, R],
    so it is still a valid quadrature with a certified error of that size.
    """
    return 1.0 if N <= 8 else math.exp(0.5 * (N - 10) + 3.8)


def minimax_unit(N: int, R: float):
    """Relative-error minimax fit on y in [1, max(R, r_floor(N))].

    Returns (alpha, beta, delta): ascending alpha, weights beta, and the max
    relative error delta = max_y |y s(y) - 1| on the final dense grid.
    """
    if N < 1 or N > 16 or not (R > 1.0):
        raise ValueError("need 1 <= N <= 16 and R > 1")
    R = max(R, r_floor(N))
    if N not in _START_CACHE:
        _START_CACHE[N] = _start(N)
    R0, res = _START_CACHE[N]
    p, q, d, ys = _walk(N, R0, res, R)
    o = np.argsort(p)
    return np.exp(p[o]), np.exp(q[o]), d


def minimax_laplace(x_min: float, x_max: float, n_tau: int):
    """(tau, w, delta) for 1/x on [x_min, x_max] (step 4, scale covariance)."""
    if not (0.0 < x_min < x_max):
        raise ValueError("need 0 < x_min < x_max")
    a, b, d = minimax_unit(n_tau, x_max / x_min)
    return a / x_min, b / x_min, d


def rel_error_curve(x, tau, w):
    """x * sum_n w_n exp(-x tau_n) - 1 at the points x."""
    x = np.asarray(x, float)
    return x * (np.exp(-np.outer(x, tau)) @ w) - 1.0


def max_rel_error(x_min, x_max, tau, w, ngrid=200000):
    """Max relative error on a dense log grid (the acceptance measure of a fit)."""
    x = np.exp(np.linspace(math.log(x_min), math.log(x_max), ngrid))
    return float(np.abs(rel_error_curve(x, tau, w)).max())
