"""The oracle against the numbers the paper prints (tests/golden/paper_constants.json)."""
import json
import math
import os

import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def g(k):
    return GOLD[k]["value"]


def test_kernel_constants(orc):
    H = 0.8
    assert orc.W(0.0, H) == pytest.approx(g("c4_prefactor_numerator") / (g("c4_prefactor_denominator_over_pi") * math.pi * H ** 3), rel=1e-15)
    # the polynomial's eta^2 coefficient: W(eta) / ((1-eta)^6 W(0)) = 1 + 6 eta + c eta^2
    for eta in (0.1, 0.37, 0.8):
        ratio = orc.W(eta * H, H) / ((1 - eta) ** 6 * orc.W(0.0, H))
        assert (ratio - 1 - 6 * eta) / eta ** 2 == pytest.approx(g("c4_eta2_coefficient"), rel=1e-9)


def test_parameter_defaults(orc):
    p = orc.params(g("Nres_standard"))
    # N_res = (4 pi / 3) n_h^3 links the two printed resolution numbers
    assert p["nh"] == pytest.approx(g("nh_standard"), rel=1e-3)
    assert p["Cl"] == g("viscosity_Cl") and p["Cq"] == g("viscosity_Cq")
    assert p["eps"] == g("viscosity_eps")
    assert p["eta_c"] * p["nh"] == pytest.approx(g("eta_crit_times_nh"))
    assert p["eta_f"] * p["nh"] == pytest.approx(g("eta_fold_times_nh"))
    assert p["gamma"] == g("gamma_monatomic")


def test_thacker_lambda(orc):
    c, o, pw = g("thacker_lambda_low")
    D = 0.7          # Delta < 1: N = N_res / Delta^3
    lam = c * (o + D ** pw)
    assert orc.thacker_step(1.0, 64.0 / D ** 3, 64.0) == pytest.approx(1 - lam + lam * D, rel=1e-14)
    c, o, pw = g("thacker_lambda_high")
    D = 1.6
    lam = c * (o + D ** pw)
    assert orc.thacker_step(1.0, 64.0 / D ** 3, 64.0) == pytest.approx(1 - lam + lam * D, rel=1e-14)
