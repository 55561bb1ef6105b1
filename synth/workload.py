"""Seeded synthetic cell states (T, p, Y) for the chemistry workloads.

The paper advances the chemistry of every LES cell of a swirl-flame mesh
(Sec. III: 5.0 M cells) over one flow step; those fields are not available.
These generators give inputs of the same kind: a block of cells crossed by a
wrinkled premixed flame sheet, with cold fuel/air on one side, burnt products
on the other and radical-rich flame-front states in between.  Only element
bookkeeping is done here (mixture composition, complete-combustion products);
no kinetics, equilibrium or integration.

Recipe (fractions are of the cell count):

* flame front, 30 %: blend of the local cold mixture and its products with a
  progress c ~ U(0.05, 0.95), plus 10^U[-3,-1.5] of mass spread over the
  non-major species (radicals); T = 1200 + 1000 c + 50 N(0,1), clipped to
  [1200, 2200] K;
* cold reactants, 35 %: fuel/air (air = O2 + 3.76 N2 by moles) at the local
  equivalence ratio phi in [0.5, 1.5], T in [300, 600] K, plus 1e-9 trace of
  every other species;
* products, 35 %: complete-combustion products of the local mixture (lean:
  CO2, H2O, O2, N2; rich: CO/H2 left over) plus 10^U[-4,-2.5] of radicals,
  T in [1800, 2400] K (near-equilibrium stand-in).

The sheet is z = Lz/2 + two seeded sinusoidal wrinkles; a cell belongs to the
front if its distance to the sheet is below 0.15 Lz.  Cells are stored
x-fastest.  ``shuffle=True`` permutes them (a stress case for binning).
"""
from __future__ import annotations

import numpy as np

from .mechanism import Mechanism, _vec

P_ATM = 101325.0


def _mole_to_mass(X, W):
    m = X * W[None, :]
    return m / m.sum(1, keepdims=True)


def _species_vec_index(mech: Mechanism, **counts):
    v = _vec(mech.elements, **counts)
    for k in range(mech.K):
        if tuple(int(x) for x in mech.composition[k]) == v:
            return k
    raise KeyError(counts)


def fuel_air_moles(mech: Mechanism, phi):
    """Mole numbers (n_cells, K) of fuel/air at equivalence ratio ``phi``."""
    phi = np.asarray(phi, np.float64)
    E = mech.elements
    fuel = _species_vec_index(mech, C=1, H=4) if "C" in E else _species_vec_index(mech, H=2)
    o2 = _species_vec_index(mech, O=2)
    n2 = _species_vec_index(mech, N=2)
    fc = mech.composition[fuel]
    n_c = fc[E.index("C")] if "C" in E else 0
    n_h = fc[E.index("H")]
    X = np.zeros((phi.size, mech.K))
    X[:, fuel] = 1.0
    X[:, o2] = (n_c + n_h / 4.0) / phi
    X[:, n2] = 3.76 * X[:, o2]
    return X


def burnt_moles(mech: Mechanism, X):
    """Complete-combustion products of mixture moles X (element bookkeeping).

    Oxygen goes first to C as CO, then to H as H2O, then CO -> CO2; leftover
    H becomes H2 and leftover O becomes O2; N becomes N2."""
    E = mech.elements
    atoms = X @ mech.composition.astype(np.float64)         # (n, E)
    nC = atoms[:, E.index("C")] if "C" in E else np.zeros(len(X))
    nH = atoms[:, E.index("H")]
    nO = atoms[:, E.index("O")]
    nN = atoms[:, E.index("N")]
    P = np.zeros_like(X)
    o_left = nO.copy()
    co = np.minimum(nC, o_left)
    o_left -= co
    h2o = np.minimum(nH / 2.0, o_left)
    o_left -= h2o
    co2 = np.minimum(co, o_left)
    o_left -= co2
    co -= co2
    P[:, _species_vec_index(mech, H=2, O=1)] += h2o
    P[:, _species_vec_index(mech, H=2)] += nH / 2.0 - h2o
    P[:, _species_vec_index(mech, O=2)] += o_left / 2.0
    P[:, _species_vec_index(mech, N=2)] += nN / 2.0
    if "C" in E:
        P[:, _species_vec_index(mech, C=1, O=2)] += co2
        P[:, _species_vec_index(mech, C=1, O=1)] += co
    return P


def _add_minor(Y, rng, frac, majors, alpha=0.7):
    """Add ``frac`` (per cell) of mass spread over non-major species, renormalise."""
    n, K = Y.shape
    minor = np.array([k for k in range(K) if k not in majors])
    w = rng.dirichlet(alpha * np.ones(minor.size), n)
    Y = Y * (1.0 - frac)[:, None]
    Y[:, minor] += frac[:, None] * w
    return Y / Y.sum(1, keepdims=True)


def uniform_cells(mech: Mechanism, n: int, seed: int, T_range=(900.0, 2400.0),
                  alpha=0.5, p=P_ATM):
    """T ~ U[T_range], Y ~ Dirichlet(alpha), p = 1 atm (the small DI workload)."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(*T_range, n)
    Y = rng.dirichlet(alpha * np.ones(mech.K), n)
    return T, np.full(n, p), Y


def flame_block(mech: Mechanism, nx: int, seed: int, shuffle: bool = False, p=P_ATM):
    """nx^3 cells crossed by a wrinkled flame sheet (x-fastest order).

    Returns T[n], p[n], Y[n, K] (float64) and the region label per cell
    (0 cold, 1 front, 2 products)."""
    rng = np.random.default_rng(seed)
    n = nx ** 3
    idx = np.arange(n)
    x = (idx % nx) / nx
    y = ((idx // nx) % nx) / nx
    z = (idx // (nx * nx)) / nx
    ph = rng.uniform(0, 2 * np.pi, 4)
    sheet = 0.5 + 0.08 * np.sin(2 * np.pi * x + ph[0]) * np.cos(2 * np.pi * y + ph[1]) \
        + 0.04 * np.sin(4 * np.pi * (x + y) + ph[2])
    d = z - sheet
    region = np.where(d < -0.15, 0, np.where(d > 0.15, 2, 1))
    phi = 1.0 + 0.45 * np.sin(2 * np.pi * y + ph[3]) * np.cos(np.pi * x) + 0.05 * rng.standard_normal(n)
    phi = np.clip(phi, 0.5, 1.5)

    W = mech.W
    Xc = fuel_air_moles(mech, phi)
    Yc = _mole_to_mass(Xc, W)
    Yb = _mole_to_mass(burnt_moles(mech, Xc), W)
    majors = set(np.nonzero(Yc.max(0) > 0)[0]) | set(np.nonzero(Yb.max(0) > 0)[0])

    T = np.empty(n)
    Y = np.empty((n, mech.K))
    c0 = region == 0
    T[c0] = 300.0 + 300.0 * np.clip(0.5 + 0.5 * np.sin(3 * x[c0] + ph[0]) * np.cos(2 * y[c0])
                                    + 0.05 * rng.standard_normal(c0.sum()), 0, 1)
    Y[c0] = _add_minor(Yc[c0], rng, np.full(c0.sum(), 1e-9 * mech.K), majors)

    c2 = region == 2
    T[c2] = rng.uniform(1800.0, 2400.0, c2.sum())
    Y[c2] = _add_minor(Yb[c2], rng, 10.0 ** rng.uniform(-4.0, -2.5, c2.sum()), majors)

    c1 = region == 1
    prog = np.clip(0.5 + (d[c1] / 0.3) + 0.1 * rng.standard_normal(c1.sum()), 0.05, 0.95)
    Ymix = (1 - prog)[:, None] * Yc[c1] + prog[:, None] * Yb[c1]
    Y[c1] = _add_minor(Ymix, rng, 10.0 ** rng.uniform(-3.0, -1.5, c1.sum()), majors)
    T[c1] = np.clip(1200.0 + 1000.0 * prog + 50.0 * rng.standard_normal(c1.sum()), 1200.0, 2200.0)

    P = np.full(n, p)
    if shuffle:
        perm = rng.permutation(n)
        T, P, Y, region = T[perm], P[perm], Y[perm], region[perm]
    return T, P, np.ascontiguousarray(Y), region


def ignition_initial_states(mech: Mechanism, n: int, seed: int,
                            phi_range=(0.5, 1.5), T0_range=(900.0, 1500.0), p=P_ATM):
    """Initial fuel/air states for 0-D constant-pressure ignition trajectories."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(*phi_range, n)
    T0 = rng.uniform(*T0_range, n)
    Y = _mole_to_mass(fuel_air_moles(mech, phi), mech.W)
    majors = set(np.nonzero(Y.max(0) > 0)[0])
    Y = _add_minor(Y, rng, np.full(n, 1e-9 * mech.K), majors)
    return T0, np.full(n, p), Y, phi


def perturb_states(T, Y, seed, y_rel=0.05, t_abs=20.0):
    """Y <- Y (1 + y_rel N(0,1)) clipped at 0 and renormalised; T <- T + t_abs N(0,1)."""
    rng = np.random.default_rng(seed)
    Yp = np.maximum(Y * (1.0 + y_rel * rng.standard_normal(Y.shape)), 0.0)
    Yp /= Yp.sum(1, keepdims=True)
    return T + t_abs * rng.standard_normal(T.shape), Yp


def element_ratios(mech: Mechanism, Y):
    """Molar H/C, O/N and elemental equivalence ratio (2 n_C + n_H / 2) / n_O of
    mass fractions Y (n, K); a ratio whose elements the mechanism lacks is NaN."""
    E = list(mech.elements)
    n = (np.asarray(Y, np.float64) / mech.W[None, :]) @ mech.composition.astype(np.float64)
    col = {e: n[:, E.index(e)] if e in E else np.zeros(len(n)) for e in ("C", "H", "O", "N")}
    with np.errstate(divide="ignore", invalid="ignore"):
        hc = col["H"] / col["C"] if "C" in E else np.full(len(n), np.nan)
        on = col["O"] / col["N"]
        phi = (2.0 * col["C"] + 0.5 * col["H"]) / col["O"]
    return np.stack([hc, on, phi], 1)


def hfrd_states(mech: Mechanism, T, p, Y, n, seed, windows, alpha=0.125, beta=10.0, theta=0.1,
                T_range=(300.0, 3000.0), max_rounds=200):
    """Random compositions around base states (T, p, Y) by the perturbation of
    the hybrid flamelet/random data recipe (paper Sec. II.B, Eqs. 3-6), each
    gamma ~ U[-1, 1] drawn per variable and state:
        T' = T + alpha gamma (T_max - T_min)
        p' = p + beta gamma (p_max - p_min)
        Y'_N2 = Y_N2 + alpha gamma (Y_N2,max - Y_N2,min)
        Y'_j = Y_j^(1 + theta gamma)   (every other species)
    with the extremes taken over the base states; the mass fractions are then
    normalised to unit sum.  A state is kept when its H/C, O/N and equivalence
    ratio lie in ``windows`` (three (lo, hi) pairs, None to skip one; see
    element_ratios) and T' in T_range; the rest are drawn again.  Returns
    (T, p, Y) of n states and the indices of their base states."""
    rng = np.random.default_rng(seed)
    n2 = _species_vec_index(mech, N=2)
    T, p, Y = np.asarray(T, np.float64), np.asarray(p, np.float64), np.asarray(Y, np.float64)
    dT, dp, dn2 = T.max() - T.min(), p.max() - p.min(), Y[:, n2].max() - Y[:, n2].min()
    outT, outP, outY, outB = [], [], [], []
    got = 0
    for _ in range(max_rounds):
        if got >= n:
            break
        m = 2 * (n - got) + 64
        b = rng.integers(0, T.size, m)
        g = rng.uniform(-1.0, 1.0, (m, 3))
        Tn = T[b] + alpha * g[:, 0] * dT
        pn = p[b] + beta * g[:, 1] * dp
        gy = rng.uniform(-1.0, 1.0, (m, mech.K))
        Yn = np.power(np.maximum(Y[b], 0.0), 1.0 + theta * gy)
        Yn[:, n2] = np.maximum(Y[b, n2] + alpha * g[:, 2] * dn2, 0.0)
        Yn /= Yn.sum(1, keepdims=True)
        r = element_ratios(mech, Yn)
        ok = (Tn >= T_range[0]) & (Tn <= T_range[1])
        for j, w in enumerate(windows):
            if w is not None:
                ok &= (r[:, j] >= w[0]) & (r[:, j] <= w[1])
        outT.append(Tn[ok]); outP.append(pn[ok]); outY.append(Yn[ok]); outB.append(b[ok])
        got += int(ok.sum())
    if got < n:
        raise RuntimeError(f"hfrd_states: {got} of {n} states inside the windows after {max_rounds} rounds")
    T2, P2, Y2, B2 = (np.concatenate(a)[:n] for a in (outT, outP, outY, outB))
    return T2, P2, np.ascontiguousarray(Y2), B2


def air_states(mech: Mechanism, n, T=300.0, p=P_ATM):
    """Ambient air (O2 + 3.76 N2 by moles) at temperature T."""
    X = np.zeros((n, mech.K))
    X[:, _species_vec_index(mech, O=2)] = 1.0
    X[:, _species_vec_index(mech, N=2)] = 3.76
    return np.full(n, T), np.full(n, p), _mole_to_mass(X, mech.W)
