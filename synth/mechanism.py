"""Seeded synthetic reaction mechanisms (input data only).

The paper's own mechanism (DRM19, 20 species / 85 reactions, Sec. II.B) is not
available, so every workload runs on a synthetic mechanism built here from a
seed.  This module only *constructs data*: element vectors, reaction lists,
Arrhenius triples and NASA-7 coefficient sets.  It evaluates none of the
kinetics, integration or property arithmetic that the oracle and the GPU
library implement; both receive the arrays produced here and nothing else.

Construction (all choices seeded through ``numpy.random.default_rng``):

* species: distinct non-zero integer element vectors with at most 5 atoms,
  always containing every single atom, O2, N2, H2, H2O, OH and the fuel
  (H2 for {H,O,N}; CH4 plus CO and CO2 for {C,H,O,N});
* reactions: atom transfers A+B <=> C+D with C = A - e_i and D = B + e_i, plus
  dissociations A+M <=> B+C with unit third-body efficiencies, so every
  reaction conserves elements by construction; the dissociation share is 1/6;
* Arrhenius: log10 A ~ U[8,14] (cgs), b ~ U[-1,2], Ea ~ U[0,60] kcal/mol;
  transfers are written in their exothermic direction and dissociations get
  Ea >= dH + 1 kcal/mol, so that reverse activation energies are non-negative;
* thermo: cp/R = c_lo + (c_hi-c_lo)(1-(1-x)^m), x = (T-300)/2700, expanded in
  powers of T (NASA-7 single range 300-3000 K), cp/R in [3.5, 6]; heats of
  formation from a bond-count model with an oxide stabilisation B_ox chosen so
  that stoichiometric fuel/air burns completely to about 2400 K;
* the stoichiometric matrix must have rank K - rank(E) (one equilibrium per
  element composition); otherwise the reaction draw is repeated.
"""
from __future__ import annotations

import itertools
import json
import math
from dataclasses import dataclass, field

import numpy as np

# Atomic masses in g/mol (conventional standard values).
ATOMIC_MASS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999}
R_U = 8.31446261815324          # J/(mol K)
CAL = 4.184                     # J/cal
T_REF = 298.15
T_LO, T_HI = 300.0, 3000.0

_FMT_ORDER = ("C", "H", "O", "N")


@dataclass
class Mechanism:
    """Flat-array mechanism description shared by the oracle and the GPU path."""

    elements: list
    element_mass: np.ndarray          # [E] g/mol
    species: list                     # names
    composition: np.ndarray           # [K, E] int32
    nasa7: np.ndarray                 # [K, 7] float64, single range
    reactants: np.ndarray             # [R, 2] int32, -1 = empty slot
    products: np.ndarray              # [R, 2] int32, -1 = empty slot
    log_A: np.ndarray                 # [R] natural log of A (cgs: cm, mol, s)
    beta: np.ndarray                  # [R]
    Ea: np.ndarray                    # [R] cal/mol
    third_body: np.ndarray            # [R] int32 (1 = "+M", unit efficiencies)
    reversible: np.ndarray            # [R] int32
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def K(self):
        return len(self.species)

    @property
    def R(self):
        return int(self.reactants.shape[0])

    @property
    def E(self):
        return len(self.elements)

    @property
    def W(self):
        """Molar masses in g/mol, from the composition (input bookkeeping)."""
        return self.composition.astype(np.float64) @ self.element_mass

    def to_json(self) -> str:
        d = {
            "elements": self.elements,
            "element_mass": self.element_mass.tolist(),
            "species": self.species,
            "composition": self.composition.tolist(),
            "nasa7": [[float(v) for v in row] for row in self.nasa7],
            "reactants": self.reactants.tolist(),
            "products": self.products.tolist(),
            "log_A": self.log_A.tolist(),
            "beta": self.beta.tolist(),
            "Ea": self.Ea.tolist(),
            "third_body": self.third_body.tolist(),
            "reversible": self.reversible.tolist(),
            "seed": self.seed,
            "meta": self.meta,
        }
        return json.dumps(d, indent=1)

    @staticmethod
    def from_json(s: str) -> "Mechanism":
        d = json.loads(s)
        return Mechanism(
            elements=d["elements"],
            element_mass=np.array(d["element_mass"], np.float64),
            species=d["species"],
            composition=np.array(d["composition"], np.int32),
            nasa7=np.array(d["nasa7"], np.float64),
            reactants=np.array(d["reactants"], np.int32),
            products=np.array(d["products"], np.int32),
            log_A=np.array(d["log_A"], np.float64),
            beta=np.array(d["beta"], np.float64),
            Ea=np.array(d["Ea"], np.float64),
            third_body=np.array(d["third_body"], np.int32),
            reversible=np.array(d["reversible"], np.int32),
            seed=d.get("seed", 0),
            meta=d.get("meta", {}),
        )

    def species_index(self, name):
        return self.species.index(name)


def species_name(vec, elements):
    parts = []
    for el in _FMT_ORDER:
        if el in elements:
            n = int(vec[elements.index(el)])
            if n == 1:
                parts.append(el)
            elif n > 1:
                parts.append(f"{el}{n}")
    return "".join(parts)


def _vec(elements, **counts):
    v = np.zeros(len(elements), np.int32)
    for el, n in counts.items():
        v[elements.index(el)] = n
    return tuple(int(x) for x in v)


def _nasa7_from_cp_curve(c_lo, c_hi, m, h_f, s298):
    """NASA-7 coefficients for cp/R = c_hi - (c_hi-c_lo)(1-x)^m, x=(T-300)/2700.

    (1-x) = u0 + u1 T with u0 = 1 + 300/2700 and u1 = -1/2700; the binomial
    expansion gives the T-power coefficients.  a6 and a7 pin h(298.15) = h_f
    and s(298.15) = s298 (both molar, SI)."""
    u0 = 1.0 + T_LO / (T_HI - T_LO)
    u1 = -1.0 / (T_HI - T_LO)
    a = np.zeros(7)
    a[0] = c_hi
    for j in range(m + 1):
        a[j] -= (c_hi - c_lo) * math.comb(m, j) * u0 ** (m - j) * u1 ** j
    t = T_REF
    h_poly = a[0] * t + a[1] * t**2 / 2 + a[2] * t**3 / 3 + a[3] * t**4 / 4 + a[4] * t**5 / 5
    s_poly = a[0] * math.log(t) + a[1] * t + a[2] * t**2 / 2 + a[3] * t**3 / 3 + a[4] * t**4 / 4
    a[5] = h_f / R_U - h_poly
    a[6] = s298 / R_U - s_poly
    return a


def _cp_curve_integral(c_lo, c_hi, m, T0, T1):
    """Integral of the generator's cp/R curve over [T0, T1] (kelvin), closed form."""
    L = T_HI - T_LO

    def prim(T):
        x = (T - T_LO) / L
        return c_hi * T + (c_hi - c_lo) * L * (1.0 - x) ** (m + 1) / (m + 1)

    return prim(T1) - prim(T0)


def generate(n_species: int, n_reactions: int, elements, seed: int,
             max_atoms: int = 5) -> Mechanism:
    """Seeded synthetic mechanism with ``n_species`` species over ``elements``."""
    elements = list(elements)
    E = len(elements)
    has_C = "C" in elements
    rng = np.random.default_rng(seed)

    required = [_vec(elements, **{el: 1}) for el in elements]
    required += [_vec(elements, H=2), _vec(elements, O=2), _vec(elements, N=2),
                 _vec(elements, H=2, O=1), _vec(elements, O=1, H=1)]
    if has_C:
        fuel = _vec(elements, C=1, H=4)
        required += [_vec(elements, C=1, O=2), _vec(elements, C=1, O=1), fuel]
    else:
        fuel = _vec(elements, H=2)
    required = list(dict.fromkeys(required))
    if len(required) > n_species:
        raise ValueError("too few species for the required set")

    all_pool = [v for n_at in range(1, max_atoms + 1)
                for v in itertools.product(range(n_at + 1), repeat=E) if sum(v) == n_at]
    all_pool = list(dict.fromkeys(tuple(int(x) for x in v) for v in all_pool))
    all_pool = [v for v in all_pool if v not in required]
    keys = rng.random(len(all_pool))
    order = sorted(range(len(all_pool)), key=lambda i: sum(all_pool[i]) + 1.5 * keys[i])
    pool_vecs = [all_pool[i] for i in order]

    for attempt in range(200):
        extra = pool_vecs[: n_species - len(required)] if attempt == 0 else \
            [pool_vecs[i] for i in sorted(rng.choice(len(pool_vecs),
                                                     n_species - len(required),
                                                     replace=False))]
        spec = required + list(extra)
        mech = _try_reactions(spec, elements, n_reactions, rng, fuel, seed)
        if mech is not None:
            return mech
    raise RuntimeError("could not draw a well-posed mechanism")


def _try_reactions(spec, elements, n_reactions, rng, fuel, seed):
    E = len(elements)
    K = len(spec)
    index = {v: k for k, v in enumerate(spec)}
    comp = np.array(spec, np.int32)
    unit = [tuple(int(i == e) for i in range(E)) for e in range(E)]

    transfers = {}
    for a, b in itertools.product(range(K), range(K)):
        for e in range(E):
            if comp[a, e] < 1:
                continue
            c_vec = tuple(int(x) for x in comp[a] - np.array(unit[e]))
            d_vec = tuple(int(x) for x in comp[b] + np.array(unit[e]))
            if sum(c_vec) == 0 or c_vec not in index or d_vec not in index:
                continue
            c, d = index[c_vec], index[d_vec]
            lhs, rhs = tuple(sorted((a, b))), tuple(sorted((c, d)))
            if lhs == rhs:
                continue
            key = frozenset((lhs, rhs))
            transfers.setdefault(key, (lhs, rhs))
    dissoc = {}
    for a in range(K):
        for b in range(K):
            for c in range(b, K):
                if np.array_equal(comp[a], comp[b] + comp[c]):
                    dissoc[(a, b, c)] = ((a,), (b, c))
    n_dis = int(round(n_reactions / 6.0))
    n_tr = n_reactions - n_dis
    tr_keys = sorted(transfers.values())
    di_keys = sorted(dissoc.values())
    if not tr_keys or not di_keys:
        return None

    def pick(keys, n):
        # distinct reactions first; a small species set cannot hold n distinct
        # ones, so the remainder are duplicates (same stoichiometry, their own
        # Arrhenius triple), as real mechanisms mark with DUPLICATE
        if len(keys) >= n:
            return [keys[i] for i in sorted(rng.choice(len(keys), n, replace=False))]
        extra = rng.choice(len(keys), n - len(keys), replace=True)
        return list(keys) + [keys[i] for i in sorted(extra)]

    sel_tr = pick(tr_keys, n_tr)
    sel_di = pick(di_keys, n_dis)
    rxns = [(l, r, 0) for l, r in sel_tr] + [(l, r, 1) for l, r in sel_di]

    nu = np.zeros((K, len(rxns)))
    for j, (l, r, _) in enumerate(rxns):
        for s in l:
            nu[s, j] -= 1
        for s in r:
            nu[s, j] += 1
    rank_E = np.linalg.matrix_rank(comp.astype(np.float64))
    if np.linalg.matrix_rank(nu) != K - rank_E:
        return None

    # ---- thermochemistry ------------------------------------------------
    D = 100.0 * 1000 * CAL       # J/mol per bond
    atoms = comp.sum(1)
    u = rng.uniform(-1, 1, K)
    refs = {_vec(elements, H=2), _vec(elements, O=2), _vec(elements, N=2)}
    for k, v in enumerate(spec):
        if v in refs:
            u[k] = 0.0
    iO = elements.index("O")
    iH = elements.index("H")
    nC = comp[:, elements.index("C")] if "C" in elements else np.zeros(K, np.int32)
    n_ob = np.minimum(comp[:, iO], comp[:, iH] + 2 * nC)
    base_hf = atoms * D / 2 - D * (atoms - 1) * (1 + 0.3 * u)
    s298 = R_U * (10.0 + 3.0 * atoms + rng.uniform(-1, 1, K))
    s298[[index[v] for v in refs if v in index]] = R_U * (10.0 + 3.0 * 2)
    c_lo = 3.5 + 0.25 * rng.random(K)
    c_hi = np.minimum(6.0, c_lo + 0.4 * (atoms - 1) + 0.3 * rng.random(K) + 0.1)
    m_exp = rng.choice([2, 3, 4], K)

    # B_ox: stoichiometric fuel/air burns completely (CO2, H2O) to 2400 K.
    f = index[fuel]
    fc = comp[f]
    n_c = fc[elements.index("C")] if "C" in elements else 0
    n_h = fc[iH]
    o2 = index[_vec(elements, O=2)]
    n2 = index[_vec(elements, N=2)]
    h2o = index[_vec(elements, H=2, O=1)]
    react = {f: 1.0, o2: n_c + n_h / 4.0, n2: 3.76 * (n_c + n_h / 4.0)}
    prod = {h2o: n_h / 2.0, n2: 3.76 * (n_c + n_h / 4.0)}
    if n_c:
        prod[index[_vec(elements, C=1, O=2)]] = float(n_c)
    sens = sum(n * R_U * _cp_curve_integral(c_lo[k], c_hi[k], m_exp[k], T_REF, 2400.0)
               for k, n in prod.items())
    dh0 = sum(n * base_hf[k] for k, n in prod.items()) - sum(n * base_hf[k] for k, n in react.items())
    dob = sum(n * n_ob[k] for k, n in prod.items()) - sum(n * n_ob[k] for k, n in react.items())
    b_ox = (sens + dh0) / dob
    if not (0.0 < b_ox < 4 * D):
        return None
    h_f = base_hf - b_ox * n_ob

    nasa = np.array([_nasa7_from_cp_curve(c_lo[k], c_hi[k], int(m_exp[k]), h_f[k], s298[k])
                     for k in range(K)])

    # ---- Arrhenius, written in the exothermic direction ---------------------
    R = len(rxns)
    reac = -np.ones((R, 2), np.int32)
    prodm = -np.ones((R, 2), np.int32)
    log10A = rng.uniform(8.0, 14.0, R)
    beta = rng.uniform(-1.0, 2.0, R)
    Ea = rng.uniform(0.0, 60.0, R) * 1000.0      # cal/mol
    tb = np.zeros(R, np.int32)
    for j, (l, r, is_dis) in enumerate(rxns):
        dh = (sum(h_f[s] for s in r) - sum(h_f[s] for s in l)) / CAL   # cal/mol
        if is_dis:
            tb[j] = 1
            Ea[j] = max(Ea[j], dh + 1000.0)
        elif dh > 0:
            l, r = r, l
        for i, s in enumerate(l):
            reac[j, i] = s
        for i, s in enumerate(r):
            prodm[j, i] = s
    names = [species_name(v, elements) for v in spec]
    return Mechanism(
        elements=list(elements),
        element_mass=np.array([ATOMIC_MASS[e] for e in elements]),
        species=names,
        composition=comp,
        nasa7=nasa,
        reactants=reac,
        products=prodm,
        log_A=log10A * math.log(10.0),
        beta=beta,
        Ea=Ea,
        third_body=tb,
        reversible=np.ones(R, np.int32),
        seed=seed,
        meta={"fuel": species_name(fuel, elements), "B_ox_J_per_mol": float(b_ox),
              "h_f_J_per_mol": h_f.tolist(), "s298_J_per_molK": s298.tolist(),
              "cp_curve": [[float(c_lo[k]), float(c_hi[k]), int(m_exp[k])] for k in range(K)]},
    )


# Mechanisms of the three workload families.
def mech_small(seed: int = 1009) -> Mechanism:
    """9 species / 24 reactions over {H,O,N}."""
    return generate(9, 24, ["H", "O", "N"], seed)


def mech_medium(seed: int = 1032) -> Mechanism:
    """32 species / 160 reactions over {C,H,O,N}."""
    return generate(32, 160, ["C", "H", "O", "N"], seed)


def mech_large(seed: int = 1053) -> Mechanism:
    """53 species / 325 reactions over {C,H,O,N}."""
    return generate(53, 325, ["C", "H", "O", "N"], seed)


def custom(elements, composition, nasa7, reactions, names=None, element_mass=None) -> Mechanism:
    """Hand-written mechanism for closed-form tests.

    ``reactions`` is a list of (reactants, products, ln_A, beta, Ea_cal, third_body,
    reversible) with species given as index tuples."""
    R = len(reactions)
    reac = -np.ones((R, 2), np.int32)
    prod = -np.ones((R, 2), np.int32)
    lnA = np.zeros(R)
    b = np.zeros(R)
    Ea = np.zeros(R)
    tb = np.zeros(R, np.int32)
    rv = np.zeros(R, np.int32)
    for j, (l, r, la, bb, ea, t, rev) in enumerate(reactions):
        reac[j, :len(l)] = l
        prod[j, :len(r)] = r
        lnA[j], b[j], Ea[j], tb[j], rv[j] = la, bb, ea, t, rev
    comp = np.array(composition, np.int32)
    em = np.array(element_mass if element_mass is not None
                  else [ATOMIC_MASS.get(e, 1.0) for e in elements], np.float64)
    return Mechanism(list(elements), em,
                     names or [f"S{k}" for k in range(comp.shape[0])],
                     comp, np.array(nasa7, np.float64), reac, prod, lnA, b, Ea, tb, rv)
