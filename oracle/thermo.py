"""Equation-of-state helpers for the multiphase workloads.

TEST INFRASTRUCTURE ONLY (used by the tests to pin initial densities).

Maxwell construction (Section 5.4 starts liquid and gas at the coexistence
densities given by the equal-area rule): at temperature T the
coexisting densities satisfy equal pressure and equal chemical potential,
p(rho_g) = p(rho_l) and mu(rho_g) = mu(rho_l), where mu = integral dp / rho is
the isothermal chemical potential.
"""
import math

import numpy as np


def vdw_pressure(rho, a, b, T):
    """van der Waals EOS p = rho T / (1 - b rho) - a rho^2."""
    return rho * T / (1.0 - b * rho) - a * rho * rho


def vdw_mu(rho, a, b, T):
    """Chemical potential of the van der Waals gas up to a T-dependent constant:
    mu = T [ln(rho / (1 - b rho)) + 1 / (1 - b rho)] - 2 a rho (integral of dp/rho)."""
    return T * (math.log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * a * rho


def vdw_critical(a, b):
    """Critical point rho_c = 1/(3b), T_c = 8a/(27b)."""
    return 1.0 / (3.0 * b), 8.0 * a / (27.0 * b)


def vdw_spinodal(a, b, T):
    """Densities where dp/drho = T/(1 - b rho)^2 - 2 a rho = 0 (gas side, liquid side)."""
    rc, _ = vdw_critical(a, b)
    dp = lambda r: T / (1.0 - b * r) ** 2 - 2.0 * a * r

    def bisect(lo, hi):
        flo = dp(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if (dp(mid) > 0) == (flo > 0):
                lo, flo = mid, dp(mid)
            else:
                hi = mid
        return 0.5 * (lo + hi)

    return bisect(1e-9, rc), bisect(rc, (1.0 - 1e-12) / b)


def vdw_maxwell(a, b, T, tol=1e-14, maxit=100):
    """Coexisting (rho_g, rho_l) by Newton on [p_g - p_l, mu_g - mu_l] = 0."""
    sg, sl = vdw_spinodal(a, b, T)
    rg, rl = 0.5 * sg, min(0.5 * (sl + 1.0 / b), sl + 0.5 * (1.0 / b - sl))
    for _ in range(maxit):
        p = lambda r: vdw_pressure(r, a, b, T)
        dp = lambda r: T / (1.0 - b * r) ** 2 - 2.0 * a * r
        f = np.array([p(rg) - p(rl), vdw_mu(rg, a, b, T) - vdw_mu(rl, a, b, T)])
        J = np.array([[dp(rg), -dp(rl)], [dp(rg) / rg, -dp(rl) / rl]])
        d = np.linalg.solve(J, -f)
        rg_new, rl_new = rg + d[0], rl + d[1]
        rg = min(max(rg_new, 0.5 * rg), sg)
        rl = max(min(rl_new, 0.5 * (rl + 1.0 / b)), sl)
        if abs(d[0]) < tol * rg and abs(d[1]) < tol * rl:
            break
    return rg, rl


# ------------------------------------------------------ Carnahan-Starling


def cs_pressure(rho, a, b, T):
    """Carnahan-Starling EOS of Section 5.4, Eq. (5.9), with R_g = 1:
    p = rho T (1 + e + e^2 - e^3) / (1 - e)^3 - a rho^2, e = b rho / 4."""
    e = 0.25 * b * rho
    return rho * T * (1.0 + e + e * e - e ** 3) / (1.0 - e) ** 3 - a * rho * rho


def cs_dpdrho(rho, a, b, T):
    """dp/drho = T (1 + 4e + 4e^2 - 4e^3 + e^4) / (1 - e)^4 - 2 a rho."""
    e = 0.25 * b * rho
    return T * (1.0 + 4.0 * e + 4.0 * e * e - 4.0 * e ** 3 + e ** 4) / (1.0 - e) ** 4 - 2.0 * a * rho


def cs_mu(rho, a, b, T):
    """Chemical potential up to a T-dependent constant, mu = integral dp / rho:
    T [ln rho + (8e - 9e^2 + 3e^3) / (1 - e)^3] - 2 a rho."""
    e = 0.25 * b * rho
    return T * (math.log(rho) + (8.0 * e - 9.0 * e * e + 3.0 * e ** 3) / (1.0 - e) ** 3) - 2.0 * a * rho


def cs_critical(a, b):
    """Critical point: the largest T at which dp/drho touches zero, i.e. the
    maximum over rho of 2 a rho (1 - e)^4 / (1 + 4e + 4e^2 - 4e^3 + e^4)
    (golden-section search on e in (0, 1))."""
    def tstar(e):
        return 2.0 * a * (4.0 * e / b) * (1.0 - e) ** 4 / (1.0 + 4.0 * e + 4.0 * e * e - 4.0 * e ** 3 + e ** 4)
    lo, hi = 1e-6, 0.5
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(200):
        m1, m2 = hi - gr * (hi - lo), lo + gr * (hi - lo)
        if tstar(m1) < tstar(m2):
            lo = m1
        else:
            hi = m2
    e = 0.5 * (lo + hi)
    return 4.0 * e / b, tstar(e)


def cs_spinodal(a, b, T):
    """Densities where dp/drho = 0 (gas side, liquid side), T < Tc."""
    rc, _ = cs_critical(a, b)
    dp = lambda r: cs_dpdrho(r, a, b, T)

    def bisect(lo, hi):
        flo = dp(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if (dp(mid) > 0) == (flo > 0):
                lo, flo = mid, dp(mid)
            else:
                hi = mid
        return 0.5 * (lo + hi)

    return bisect(1e-12, rc), bisect(rc, (1.0 - 1e-9) * 4.0 / b)


def cs_maxwell(a, b, T, tol=1e-14, maxit=200):
    """Coexisting (rho_g, rho_l) by Newton on [p_g - p_l, mu_g - mu_l] = 0."""
    sg, sl = cs_spinodal(a, b, T)
    rg, rl = 0.3 * sg, sl + 0.5 * (4.0 / b - sl) * 0.5
    for _ in range(maxit):
        f = np.array([cs_pressure(rg, a, b, T) - cs_pressure(rl, a, b, T),
                      cs_mu(rg, a, b, T) - cs_mu(rl, a, b, T)])
        dg, dl = cs_dpdrho(rg, a, b, T), cs_dpdrho(rl, a, b, T)
        J = np.array([[dg, -dl], [dg / rg, -dl / rl]])
        d = np.linalg.solve(J, -f)
        # damped: stay strictly inside the stable branches
        rg = min(max(rg + d[0], 0.5 * rg), 0.5 * (rg + sg))
        rl = max(min(rl + d[1], 0.5 * (rl + 4.0 / b)), 0.5 * (rl + sl))
        if abs(d[0]) < tol * rg and abs(d[1]) < tol * rl:
            break
    return rg, rl
