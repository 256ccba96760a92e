"""The SLP step of Sec. 4 (plain definitions).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* LP subproblem (Sec. 4.1, problem (Pstar)) for the topology problem's single
  linear constraint, the volume (Sec. 3.4: its gradient a = W^T v > 0 is
  constant):
      min g^T s   s.t.  a^T s = b,   l <= s <= u,
  with l_i = max(-delta, x_l - x_i), u_i = min(delta, x_u - x_i) and
  b = -c(x) = V_max - a^T x.  Reading: the volume constraint is taken as an
  equality, the form of problem (P).  With one constraint and a box the LP is
  a fractional knapsack: start from s = l, and raise the variables in order of
  the ratio r_i = -g_i / a_i (objective decrease per unit of volume), highest
  first, each to its upper bound, until the volume budget B = b - a^T l is
  used up; the variable that crosses the budget is raised partially.  Ties in
  r are taken in increasing index order (any order gives the same objective).
  The multiplier of the equality is the critical ratio lambda = r_k (the
  Lagrangian g + lambda a is <= 0 on the raised variables, >= 0 on the rest;
  the critical variable is the first, in the order, with positive capacity
  u - l whose running capacity reaches B).
* Infeasible LP (B < 0 or B above the total capacity, beyond the rounding
  allowance 2 n eps (sum |a_i l_i| + sum a_i (u_i - l_i)) of the sums that
  give them; a budget inside the allowance is clamped to the boundary): the
  artificial problem
  (Pstar2) with the box shrunk to 0.8 delta; with one constraint its solution
  is the end of the shrunk box that leaves the least violation, s = l' if
  B < 0, s = u' if B exceeds the capacity.  Reading: the upper bound of the
  shrunk box printed as max{0.8 delta; x_u - x_i} is taken as the min, the
  mirror image of the lower bound.
* Fixed design variables (Sec. 6.1) take l = u = 0, the alternative the
  paper gives to removing them from the LP.
* Step control of Algorithm 2: the predicted and actual reductions of the
  merit function psi = theta f + (1 - theta) phi, phi = |c|^2 / 2, the penalty
  parameter update (eqs. (theta1), (theta2)) and the trust-region radius
  update, in the order of the algorithm.  Reading: P_red^opt is the predicted
  reduction of f, -g^T s (printed without the minus sign), so that
  P_red = theta P_red^opt + (1 - theta) P_red^fsb as printed, and theta_sup
  is the largest theta with P_red >= P_red^fsb / 2.

Pins (tests/test_oracle_slp.py): the LP optimum against an enumeration of all
vertices of the feasible polytope on tiny instances and against scipy's
linprog on small ones (objective values; the minimiser is unique without
ties); the KKT conditions with the returned multiplier; hand-computed cases of
the theta and delta rules.
"""

import numpy as np


def lp_bounds(x, delta, xl=0.0, xu=1.0, fixed=None):
    """(l, u) of problem (Pstar); fixed variables get l = u = 0 (Sec. 6.1)."""
    x = np.asarray(x, dtype=np.float64)
    l, u = np.maximum(-delta, xl - x), np.minimum(delta, xu - x)
    if fixed is not None:
        f = np.asarray(fixed) != 0
        l, u = np.where(f, 0.0, l), np.where(f, 0.0, u)
    return l, u


def lp_step(g, a, x, b, delta, xl=0.0, xu=1.0, fixed=None):
    """Solution of the LP subproblem: (s, lambda, feasible).

    g: objective gradient, a: constraint gradient (> 0), b: right-hand side
    (a^T s = b), delta: trust-region radius, fixed: optional mask of
    variables held at s = 0 (the fixed design variables of Sec. 6.1)."""
    g = np.asarray(g, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    if np.any(a <= 0.0):
        raise ValueError("the constraint gradient must be positive")
    l, u = lp_bounds(x, delta, xl, xu, fixed)
    B = b - float(np.dot(a, l))
    cap = a * (u - l)
    # a budget within the rounding of its sums of 0 or of the capacity is the
    # boundary itself
    tau = 2 * g.size * np.finfo(np.float64).eps * (float(np.abs(a * l).sum()) + float(cap.sum()))
    if B < -tau or B > cap.sum() + tau:
        # artificial problem with the box shrunk to 0.8 delta
        l2, u2 = lp_bounds(x, 0.8 * delta, xl, xu, fixed)
        return (l2.copy() if B < 0.0 else u2.copy()), float("nan"), False
    B = min(max(B, 0.0), float(cap.sum()))
    r = -g / a
    order = sorted(range(g.size), key=lambda i: (-r[i], i))
    s = l.copy()
    left = B
    lam = None
    last = None
    for i in order:
        if cap[i] <= 0.0:
            continue  # u = l
        last = i
        if cap[i] < left:
            s[i] = u[i]
            left -= cap[i]
            continue
        # the critical variable: the first whose running capacity reaches B
        s[i] = u[i] if cap[i] == left else l[i] + left / a[i]
        lam = r[i]
        break
    if lam is None:
        # rounding left the budget above the capacity: the last variable with
        # capacity; with none at all, the first in the order
        lam = r[last] if last is not None else r[order[0]]
    return s, lam, True


def merit_reductions(theta, f0, f1, g, s, c0, c1, a):
    """(A_red, P_red, P_fsb, P_opt) of Sec. 4.1.3 for one constraint c with
    gradient a: phi = c^2 / 2, M(x, s) = (a^T s + c)^2 / 2."""
    phi0, phi1 = 0.5 * c0 * c0, 0.5 * c1 * c1
    m0, m1 = 0.5 * c0 * c0, 0.5 * (float(np.dot(a, s)) + c0) ** 2
    gs = float(np.dot(g, s))
    a_red = theta * (f0 - f1) + (1.0 - theta) * (phi0 - phi1)
    p_fsb = m0 - m1
    # the predicted reduction of f (printed as g^T s without the sign; with the
    # sign, P_red = theta P_opt + (1 - theta) P_fsb as printed for P_red)
    p_opt = -gs
    p_red = -theta * gs + (1.0 - theta) * p_fsb
    return a_red, p_red, p_fsb, p_opt


def theta_update(k, theta_hist, theta_max, p_fsb, p_opt, N=1e6):
    """theta_k = min(theta_large, theta_sup, theta_max), eqs. (theta1), (theta2);
    theta_hist holds theta_0 .. theta_{k-1}."""
    large = (1.0 + N / (k + 1) ** 1.1) * min(theta_hist)
    if p_opt <= 0.5 * p_fsb:
        sup = 0.5 * p_fsb / (p_fsb - p_opt)
    else:
        sup = 1.0
    return min(large, sup, theta_max)


def trust_update(a_red, p_red, delta, s_inf, box_inf, delta_min):
    """(accepted, new delta) of Algorithm 2."""
    if a_red < 0.1 * p_red:
        return False, min(0.25 * s_inf, 0.1 * delta)
    d = delta
    if a_red >= 0.5 * p_red:
        d = min(2.0 * delta, box_inf)
    return True, max(d, delta_min)


def projected_gradient(x, g, a, lam, xl=0.0, xu=1.0):
    """g_P = P_X(x - (g + lambda a)) - x of the stopping test (Sec. 4.2.1)."""
    x = np.asarray(x, dtype=np.float64)
    return np.clip(x - (np.asarray(g) + lam * np.asarray(a)), xl, xu) - x


__all__ = ["lp_bounds", "lp_step", "merit_reductions", "theta_update", "trust_update",
           "projected_gradient"]
