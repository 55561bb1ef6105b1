"""FP64 reference of the steps around the chemistry advance -- TEST
INFRASTRUCTURE ONLY (only tests/, smoke() and bench.py's CPU baseline use it).

Transport properties (Sec. II.A: properties from temperature polynomials):
species viscosity and conductivity as ln(prop) = sum_j c_j (ln T)^j, j < 4,
mixture viscosity by Wilke's rule and mixture conductivity by the average of
Mathur, Tondon and Saxena.  The PaSR closure (Sec. III: the source term of
the partially stirred reactor, with the chemical time from the slowest
species formation rate and the mixing time the geometric mean of the
sub-grid (Taylor-like) and Kolmogorov times).  Readings where the text is
silent:

* the chemistry step's source is omega_k = rho (Y1_k - Y0_k) / dt with rho the
  density of the state at the step's start;
* tau_c = max over species with omega_k > 0 and Y1_k >= y_min of
  rho Y1_k / omega_k (the slowest formation; trace species below y_min are
  left out); no such species: the cell reacts not at all and kappa = 1;
* the sub-grid velocity u' = sqrt(2 k / 3), tau_Delta = Delta / u',
  epsilon = C_eps k^(3/2) / Delta (C_eps = 1.048, the one-equation sub-grid
  model's constant), tau_K = sqrt(nu / epsilon) with nu = mu / rho,
  tau_mix = sqrt(tau_Delta tau_K);
* kappa = tau_c / (tau_c + tau_mix), the closed source kappa omega_k and the
  blended state Y0 + kappa (Y1 - Y0).
"""
from __future__ import annotations

import numpy as np

R_U = 8.31446261815324
C_EPS = 1.048
Y_MIN = 1e-6


def poly_ln(coef, T):
    """exp(sum_j coef[..., j] (ln T)^j): coef [K, 4] -> values [n, K]."""
    lt = np.log(np.asarray(T, np.float64))[:, None]
    c = np.asarray(coef, np.float64)
    return np.exp(c[None, :, 0] + c[None, :, 1] * lt + c[None, :, 2] * lt ** 2 + c[None, :, 3] * lt ** 3)


def mole_fractions(Y, W_g):
    n = np.asarray(Y, np.float64) / np.asarray(W_g, np.float64)[None, :]
    return n / n.sum(1, keepdims=True)


def wilke(X, mu, W_g):
    """Mixture viscosity: sum_i X_i mu_i / sum_j X_j Phi_ij with
    Phi_ij = (1 + (mu_i/mu_j)^(1/2) (W_j/W_i)^(1/4))^2 / (8 (1 + W_i/W_j))^(1/2)."""
    X, mu, W = (np.asarray(a, np.float64) for a in (X, mu, W_g))
    n, K = X.shape
    out = np.empty(n)
    for c in range(n):
        s = 0.0
        for i in range(K):
            den = 0.0
            for j in range(K):
                phi = (1.0 + np.sqrt(mu[c, i] / mu[c, j]) * (W[j] / W[i]) ** 0.25) ** 2 / np.sqrt(8.0 * (1.0 + W[i] / W[j]))
                den += X[c, j] * phi
            s += X[c, i] * mu[c, i] / den
        out[c] = s
    return out


def mathur_saxena(X, lam):
    """Mixture conductivity: (sum_k X_k lam_k + 1 / sum_k (X_k / lam_k)) / 2."""
    X, lam = np.asarray(X, np.float64), np.asarray(lam, np.float64)
    return 0.5 * ((X * lam).sum(1) + 1.0 / (X / lam).sum(1))


def transport(mu_coef, lam_coef, W_g, T, Y):
    """(mixture viscosity [Pa s], mixture conductivity [W/(m K)]) per cell."""
    X = mole_fractions(Y, W_g)
    return wilke(X, poly_ln(mu_coef, T), W_g), mathur_saxena(X, poly_ln(lam_coef, T))


def density(W_g, T, p, Y):
    """Ideal-gas density [kg/m^3]."""
    Wbar = 1.0 / (np.asarray(Y, np.float64) / (np.asarray(W_g, np.float64) * 1e-3)[None, :]).sum(1)
    return np.asarray(p, np.float64) * Wbar / (R_U * np.asarray(T, np.float64))


def pasr(W_g, T, p, Y0, Y1, dt, k_sgs, delta, mu, c_eps=C_EPS, y_min=Y_MIN):
    """PaSR closure of one step (the readings above): returns (kappa [n],
    closed source kappa omega [n, K] in kg/(m^3 s), blended Y [n, K])."""
    Y0, Y1 = np.asarray(Y0, np.float64), np.asarray(Y1, np.float64)
    rho = density(W_g, T, p, Y0)
    omega = rho[:, None] * (Y1 - Y0) / dt
    n = Y0.shape[0]
    kappa = np.ones(n)
    for c in range(n):
        taus = [rho[c] * Y1[c, k] / omega[c, k] for k in range(Y0.shape[1])
                if omega[c, k] > 0.0 and Y1[c, k] >= y_min]
        if not taus:
            continue
        tau_c = max(taus)
        k = float(k_sgs[c])
        if k <= 0.0:
            kappa[c] = 0.0
            continue
        up = np.sqrt(2.0 * k / 3.0)
        tau_d = float(delta[c]) / up
        eps = c_eps * k ** 1.5 / float(delta[c])
        tau_k = np.sqrt(float(mu[c]) / rho[c] / eps)
        tau_mix = np.sqrt(tau_d * tau_k)
        kappa[c] = tau_c / (tau_c + tau_mix)
    return kappa, kappa[:, None] * omega, Y0 + kappa[:, None] * (Y1 - Y0)
