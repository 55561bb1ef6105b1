"""Hand-written mechanisms with closed-form behaviour, for the oracle's pins."""
import math

import numpy as np

from synth.mechanism import custom

LN10 = math.log(10.0)


def const_cp_nasa(c, a6, a7):
    """NASA-7 row with constant cp/R = c: h/RT = c + a6/T, s/R = c ln T + a7."""
    return [c, 0.0, 0.0, 0.0, 0.0, a6, a7]


def isomers(reversible, s_gap=0.0, lnA=math.log(1e13), Ea=5000.0):
    """Two isomers A, B of composition H2 (equal enthalpy), A + M -> B + M."""
    nasa = [const_cp_nasa(3.5, -1000.0, 5.0), const_cp_nasa(3.5, -1000.0, 5.0 + s_gap)]
    return custom(["H"], [[2], [2]], nasa, [((0,), (1,), lnA, 0.0, Ea, 1, int(reversible))],
                  names=["A", "B"])


def bimolecular():
    """H2 + O -> H + OH, irreversible, equal constant cp, zero reaction enthalpy."""
    nasa = [const_cp_nasa(3.5, 100.0, 2.0),      # H2
            const_cp_nasa(3.5, 300.0, 3.0),      # O
            const_cp_nasa(3.5, 150.0, 4.0),      # H
            const_cp_nasa(3.5, 250.0, 5.0)]      # OH: 150 + 250 = 100 + 300
    return custom(["H", "O"], [[2, 0], [0, 1], [1, 0], [1, 1]], nasa,
                  [((0, 1), (2, 3), math.log(3e12), 0.5, 4000.0, 0, 0)],
                  names=["H2", "O", "H", "OH"])


def tiny_hox():
    """5 species over {H, O}, mild rates, reversible (brute-force RK4 pin)."""
    R = 8.31446261815324
    # a6 from heats of formation h_f (J/mol) at 298.15 with constant cp/R
    def row(cpR, hf, s298):
        a6 = hf / R - cpR * 298.15
        a7 = s298 / R - cpR * math.log(298.15)
        return const_cp_nasa(cpR, a6, a7)
    nasa = [row(2.5, 218e3, 114.7),   # H
            row(2.5, 249e3, 161.1),   # O
            row(3.5, 0.0, 130.7),     # H2
            row(3.6, 0.0, 205.1),     # O2
            row(3.6, 39e3, 183.7)]    # OH
    comp = [[1, 0], [0, 1], [2, 0], [0, 2], [1, 1]]
    rx = [((2, 1), (0, 4), 10.0 * LN10, 0.0, 12000.0, 0, 1),   # H2 + O = H + OH
          ((3, 0), (1, 4), 10.5 * LN10, 0.0, 16000.0, 0, 1),   # O2 + H = O + OH
          ((2, 3), (4, 4), 9.0 * LN10, 0.0, 30000.0, 0, 1),    # H2 + O2 = OH + OH
          ((2,), (0, 0), 14.0 * LN10, 0.0, 80000.0, 1, 1)]     # H2 + M = H + H + M
    return custom(["H", "O"], comp, nasa, rx, names=["H", "O", "H2", "O2", "OH"])
