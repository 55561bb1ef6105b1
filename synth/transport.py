"""Seeded synthetic transport data for the synthetic mechanisms (input data only).

The paper updates transport properties with high-order temperature polynomials
(Sec. II.A, "update thermal and transport properties"); its DRM19 transport
file is not available.  This module builds, per species, the coefficients of
ln mu_k and ln lambda_k as cubic polynomials in ln T over 300-3000 K, the form
the property kernels and the oracle evaluate.  The data come from kinetic
theory with Lennard-Jones parameters assigned by atom count:

* sigma_k [Angstrom] = 2.55 + 0.42 (n_atoms - 1)^0.7 and
  eps_k / k_B [K] = 80 + 95 (n_atoms - 1)^0.6 (a smooth stand-in for tabulated
  Lennard-Jones parameters; diatomics land near N2's 3.6 A / 98 K scale);
* Chapman-Enskog viscosity mu = 2.6693e-6 sqrt(W T) / (sigma^2 Omega22(T*))
  [Pa s, W in g/mol, T* = T k_B / eps], Omega22 by the fit of Neufeld, Janzen
  and Aziz (J. Chem. Phys. 57, 1100, 1972);
* conductivity by the modified Eucken relation lambda = mu (cp + 5 R / (4 W))
  [W/(m K)], cp per unit mass from the species' NASA-7 polynomial.

Nothing here is used at run time by the kernels or the oracle other than the
coefficient arrays it returns.
"""
from __future__ import annotations

import numpy as np

from .mechanism import Mechanism, R_U, T_LO, T_HI


def lennard_jones(mech: Mechanism):
    """(sigma [Angstrom], eps/k_B [K]) per species from its atom count."""
    na = mech.composition.sum(1).astype(np.float64)
    sigma = 2.55 + 0.42 * np.power(np.maximum(na - 1.0, 0.0), 0.7)
    eps = 80.0 + 95.0 * np.power(np.maximum(na - 1.0, 0.0), 0.6)
    return sigma, eps


def omega22(Ts):
    """Reduced collision integral Omega(2,2)* (Neufeld, Janzen and Aziz 1972)."""
    Ts = np.asarray(Ts, np.float64)
    return 1.16145 * Ts ** -0.14874 + 0.52487 * np.exp(-0.77320 * Ts) + 2.16178 * np.exp(-2.43787 * Ts)


def viscosity_ce(W_g, sigma, eps, T):
    """Chapman-Enskog viscosity [Pa s] of a pure gas."""
    T = np.asarray(T, np.float64)
    return 2.6693e-6 * np.sqrt(W_g * T) / (sigma ** 2 * omega22(T / eps))


def _cp_mass(nasa, W_g, T):
    T = np.asarray(T, np.float64)
    cpR = nasa[0] + nasa[1] * T + nasa[2] * T ** 2 + nasa[3] * T ** 3 + nasa[4] * T ** 4
    return cpR * R_U / (W_g * 1e-3)


def transport_fits(mech: Mechanism, n_fit=200):
    """Coefficients [K, 4] of ln mu_k and ln lambda_k as polynomials in ln T
    (ascending powers) least-squares fitted on n_fit temperatures spaced
    evenly in ln T over 300-3000 K."""
    W = mech.composition.astype(np.float64) @ np.asarray(mech.element_mass, np.float64)
    sigma, eps = lennard_jones(mech)
    T = np.exp(np.linspace(np.log(T_LO), np.log(T_HI), n_fit))
    lt = np.log(T)
    V = np.stack([lt ** j for j in range(4)], 1)
    mu_c = np.empty((mech.K, 4))
    lam_c = np.empty((mech.K, 4))
    for k in range(mech.K):
        mu = viscosity_ce(W[k], sigma[k], eps[k], T)
        lam = mu * (_cp_mass(mech.nasa7[k], W[k], T) + 1.25 * R_U / (W[k] * 1e-3))
        mu_c[k] = np.linalg.lstsq(V, np.log(mu), rcond=None)[0]
        lam_c[k] = np.linalg.lstsq(V, np.log(lam), rcond=None)[0]
    return mu_c, lam_c
