"""Gibbs-minimisation equilibrium for the oracle's tests -- TEST INFRASTRUCTURE ONLY.

Ideal-gas equilibrium at fixed (T, p) by the element-potential method: at the
minimum of G subject to element conservation, every species obeys
    ln x_k = sum_e lambda_e a_ek - g_k/RT - ln(p/p0),
with the Lagrange multipliers lambda_e and the total mole number as unknowns
(element balances plus sum x_k = 1), solved by damped Newton.  HP equilibrium
wraps a safeguarded Newton/bisection in T around it so that the mixture
enthalpy matches h0.  G is convex for ideal gases, so the answer is unique.
Species thermochemistry comes from the oracle's NASA-7 evaluation.
"""
from __future__ import annotations

import numpy as np

P0 = 101325.0


def equilibrium_TP(om, T, p, b, x0=None, tol=1e-14, max_iter=200):
    """Mole numbers n_k (per unit of the element amounts b[E]) at (T, p)."""
    cpR, hRT, sR = om.species_thermo(T)
    g = hRT - sR
    A = om.src.composition.astype(np.float64)          # (K, E)
    K, E = A.shape
    c = -g - np.log(p / P0)
    # initial multipliers: least squares fit of a starting composition
    if x0 is None:
        x0 = np.full(K, 1.0 / K)
    lx0 = np.log(np.maximum(x0, 1e-30))
    lam = np.linalg.lstsq(A, lx0 - c, rcond=None)[0]
    nu = np.log(max(b.sum(), 1e-300))
    for it in range(max_iter):
        lx = np.clip(A @ lam + c, -700, 700)
        x = np.exp(lx)
        n = x * np.exp(nu)
        F = np.concatenate([A.T @ n - b, [x.sum() - 1.0]])
        Jm = np.zeros((E + 1, E + 1))
        Jm[:E, :E] = (A.T * n) @ A
        Jm[:E, E] = A.T @ n
        Jm[E, :E] = A.T @ x
        try:
            d = np.linalg.solve(Jm, -F)
        except np.linalg.LinAlgError:
            d = np.linalg.lstsq(Jm, -F, rcond=None)[0]
        s = 1.0
        mx = np.abs(d).max()
        if mx > 2.0:
            s = 2.0 / mx
        lam += s * d[:E]
        nu += s * d[E]
        if mx < tol and s == 1.0:
            break
    lx = A @ lam + c
    return np.exp(lx) * np.exp(nu)


def element_moles(om, Y):
    """Moles of each element per kg of mixture (Y mass fractions)."""
    A = om.src.composition.astype(np.float64)
    return (Y / (om.W * 1e-3)) @ A


def equilibrium_HP(om, h0, p, Y_in, T_guess=2000.0):
    """Equilibrium (T, Y) with mixture enthalpy h0 [J/kg] at pressure p."""
    b = element_moles(om, Y_in)
    x0 = (Y_in / om.W) / (Y_in / om.W).sum()

    def state(T):
        n = equilibrium_TP(om, T, p, b, x0=np.maximum(x0, 1e-12))
        Y = n * om.W * 1e-3
        Y /= Y.sum()
        cp, h = om.cp_h(T, Y)
        return Y, h

    lo, hi = 300.0, 4000.0
    T = T_guess
    for it in range(100):
        Y, h = state(T)
        if abs(h - h0) <= 1e-13 * max(abs(h0), 1.0):
            break
        if h < h0:
            lo = T
        else:
            hi = T
        Y2, h2 = state(T + 1e-3)
        cpe = (h2 - h) / 1e-3
        Tn = T - (h - h0) / cpe
        if not (lo < Tn < hi):
            Tn = 0.5 * (lo + hi)
        if abs(Tn - T) < 1e-11 * T:
            T = Tn
            break
        T = Tn
    Y, h = state(T)
    return T, Y
