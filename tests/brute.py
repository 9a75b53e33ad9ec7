"""Independent high-precision references used to pin the oracle.

Nothing here shares code with the oracle: these are separate derivations of
the same quantities, in 50-digit decimal arithmetic or by a different
characterisation of the solution.

* ``mbar_decimal``: the MBAR free energies as the minimiser of the convex
  objective F(f) = sum_n log sum_k N_k exp(f_k - u_kn) - sum_k N_k f_k,
  found by damped Newton in 50-digit ``decimal`` arithmetic (tiny K, N).
* ``bar_bisection``: for two states, Bennett's acceptance-ratio equation
  sum_{n in 0} 1/(1 + (N0/N1) e^{du_n - df}) = sum_{n in 1} 1/(1 + (N1/N0) e^{df - du_n})
  with du = u_1 - u_0, solved for df = f_1 - f_0 by bisection (it is
  monotone in df) with exactly rounded sums (math.fsum).
"""
from __future__ import annotations

import math
from decimal import Decimal, getcontext


def _dexp(x: Decimal) -> Decimal:
    return x.exp()


def _dlog(x: Decimal) -> Decimal:
    return x.ln()


def mbar_decimal(u, Nk, digits=50, iters=200):
    """Return f (list of float, f_0 = 0) minimising F in ``digits``-digit arithmetic."""
    getcontext().prec = digits
    K = len(Nk)
    N = len(u[0])
    U = [[Decimal(repr(float(u[k][n]))) for n in range(N)] for k in range(K)]
    Ns = [Decimal(int(x)) for x in Nk]
    f = [Decimal(0)] * K

    def terms(fv):
        # e_kn = N_k exp(f_k - u_kn) for sampled states
        D = []
        E = []
        for n in range(N):
            col = [Ns[k] * _dexp(fv[k] - U[k][n]) if Nk[k] > 0 else Decimal(0) for k in range(K)]
            s = sum(col, Decimal(0))
            D.append(s)
            E.append(col)
        return D, E

    def objective(fv):
        D, _ = terms(fv)
        return sum((_dlog(d) for d in D), Decimal(0)) - sum((Ns[k] * fv[k] for k in range(K)),
                                                             Decimal(0))

    free = [k for k in range(K) if Nk[k] > 0][1:]
    for _ in range(iters):
        D, E = terms(f)
        # P_nk = N_k W_nk
        P = [[E[n][k] / D[n] for k in range(K)] for n in range(N)]
        g = [sum((P[n][i] for n in range(N)), Decimal(0)) - Ns[i] for i in range(K)]
        H = [[(sum((P[n][i] for n in range(N)), Decimal(0)) if i == j else Decimal(0))
              - sum((P[n][i] * P[n][j] for n in range(N)), Decimal(0)) for j in range(K)]
             for i in range(K)]
        m = len(free)
        if m == 0:
            break
        A = [[H[a][b] for b in free] + [-g[a]] for a in free]
        # Gaussian elimination with partial pivoting
        for c in range(m):
            piv = max(range(c, m), key=lambda r: abs(A[r][c]))
            A[c], A[piv] = A[piv], A[c]
            for r in range(c + 1, m):
                fac = A[r][c] / A[c][c]
                for cc in range(c, m + 1):
                    A[r][cc] -= fac * A[c][cc]
        x = [Decimal(0)] * m
        for r in range(m - 1, -1, -1):
            x[r] = (A[r][m] - sum((A[r][cc] * x[cc] for cc in range(r + 1, m)), Decimal(0))) / A[r][r]
        F0 = objective(f)
        step = Decimal(1)
        while True:
            ft = list(f)
            for a, k in enumerate(free):
                ft[k] = f[k] + step * x[a]
            if objective(ft) <= F0 or step < Decimal("1e-6"):
                break
            step /= 2
        f = ft
        if max(abs(v) for v in x) < Decimal(10) ** (-(digits - 10)):
            break
    # states without samples: f_k = -log sum_n exp(-u_kn) / D_n
    D, _ = terms(f)
    for k in range(K):
        if Nk[k] == 0:
            f[k] = -_dlog(sum((_dexp(-U[k][n]) / D[n] for n in range(N)), Decimal(0)))
    f0 = f[0]
    return [float(v - f0) for v in f]


def bar_bisection(u0, u1, N0, N1, lo=-200.0, hi=200.0, iters=400):
    """df = f_1 - f_0 from Bennett's equation (samples 0..N0-1 from state 0, rest from 1)."""
    du = [b - a for a, b in zip(u0, u1)]
    d0, d1 = du[:N0], du[N0:]
    r = N0 / N1

    def h(df):
        left = math.fsum(1.0 / (1.0 + r * math.exp(x - df)) for x in d0)
        right = math.fsum(1.0 / (1.0 + math.exp(df - x) / r) for x in d1)
        return left - right  # increasing in df

    a, b = lo, hi
    for _ in range(iters):
        mid = 0.5 * (a + b)
        if h(mid) > 0:
            b = mid
        else:
            a = mid
        if b - a <= 1e-15 * max(1.0, abs(mid)):
            break
    return 0.5 * (a + b)
