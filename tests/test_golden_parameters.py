"""The paper's printed model and prior parameters (Sec. 3, stored in
tests/golden/model_parameters_sec3.json with their citation) against the
defaults of the synthetic workloads."""
import json
import os

import pytest

from synth import card_c1, card_c2, card_c3, tiny_card
from synth.cards import Prior, ALPHA_WATER, ALPHA_CEMENT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "model_parameters_sec3.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def test_prior_defaults_are_the_papers(paper):
    pr, ref = Prior(), paper["prior_simulated"]
    assert (pr.p, pr.q, pr.T, pr.sigma0, pr.m, pr.a) == (ref["p"], ref["q"], ref["T"], ref["sigma0_per_m3"],
                                                        ref["m"], ref["a"])


@pytest.mark.parametrize("mk", [card_c1, card_c2, card_c3, tiny_card])
def test_beta_is_the_papers(paper, mk):
    assert mk().array.beta == paper["forward_model"]["beta"]


def test_attenuation_reading(paper):
    """The attenuation cards take the printed water and concrete figures per MHz."""
    fm = paper["forward_model"]
    assert ALPHA_WATER == pytest.approx(fm["alpha_water_per_hz_per_m"] * 1e-6)
    assert ALPHA_CEMENT == pytest.approx(fm["alpha_concrete_per_hz_per_m"] * 1e-6)


@pytest.mark.parametrize("mk,n", [(card_c2, 50), (card_c3, 50)])
def test_iteration_counts(paper, mk, n):
    assert mk().n_iter == paper["iterations"]["simulated"] == n
