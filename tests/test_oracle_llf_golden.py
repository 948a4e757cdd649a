"""Hand-derived numerical-flux values on a two-element periodic mesh (test
infrastructure): the derivations are written out in
golden/llf_two_element.json."""
import json
import os

import numpy as np

import oracle as O
from paper_1601_07944_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "llf_two_element.json")))


def two_element_rhs(stateA, stateB, lib=None):
    mesh = W.square_mesh(1, 1.0, 0.0, 0)
    orc = O.Oracle(mesh, 2, lib=lib)
    UA = W.primitive_to_conserved(*(np.array(stateA[k]) for k in ("rho", "u", "v", "p")))
    UB = W.primitive_to_conserved(*(np.array(stateB[k]) for k in ("rho", "u", "v", "p")))
    C = np.zeros((2, 4, orc.np))
    C[0, :, 0] = UA / np.sqrt(2.0)
    C[1, :, 0] = UB / np.sqrt(2.0)
    return orc.rhs(C)


def check_cases(lib=None):
    ok = True
    c0, c1 = GOLD["cases"]
    R = two_element_rhs(c0["A"], c0["B"], lib)
    ok &= abs(R[0, 0, 0] - c0["value"]) < 1e-14
    ok &= np.all(np.abs(R[0, 1:, 0]) < 1e-14)
    ok &= abs(R[1, 0, 0] + c0["value"]) < 1e-14  # conservation: B gains what A loses
    R = two_element_rhs(c1["A"], c1["B"], lib)
    ok &= abs(R[0, 0, 0] - c1["value"]) < 1e-13
    ok &= abs(R[0, 1, 0] - c1["value_mx"]) < 1e-13
    ok &= abs(R[0, 2, 0]) < 1e-13
    ok &= abs(R[0, 3, 0] - c1["value_E"]) < 1e-13
    return bool(ok)


def test_llf_two_element_closed_form():
    assert check_cases()
