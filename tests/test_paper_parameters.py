"""The paper's printed parameters are mutually consistent (golden fixture
tests/golden/paper_parameters.json, each entry citing its paragraph)."""
import json
import os

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def load():
    with open(GOLD) as f:
        return json.load(f)


def test_splash_numbers():
    s = load()["splash"]
    we = s["rho_l"] * s["U"] ** 2 * s["D"] / s["sigma"]
    assert abs(we - s["We"]) < 1e-9
    for re, nu in zip(s["Re"], s["nu_l"]):
        assert abs(s["U"] * s["D"] / nu - re) < 1e-9
    # the rho = 0.55 contour is the phi = 1/2 level set of Eq. 4a
    assert abs(s["rho_g"] + 0.5 * (s["rho_l"] - s["rho_g"]) - s["contour_rho"]) < 1e-12
    assert s["grid"][1] * s["film_fraction"] == 15


def test_falling_numbers():
    f = load()["falling"]
    g = f["Eo"] * f["sigma"] / ((f["rho_l"] - f["rho_g"]) * f["D"] ** 2)
    assert abs(g - 8.30078125e-6) < 1e-15
    frac = f["spread_difference"] / (f["D"] / 2)
    assert abs(frac - f["spread_difference_fraction_of_R0"]) < 0.005
