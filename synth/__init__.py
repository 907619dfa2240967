"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds problem cards (plain numbers) and seeded random draws only:
phantoms, noise vectors and random test vectors.  It contains none of the
reconstruction method's arithmetic (no travel times, templates, operators or
prior terms), so the FP64 oracle and the HIP path can both consume it without
sharing any computation.
"""
from .cards import (Medium, Grid, Array, Acquisition, Prior, PhantomSpec, Card,
                    card_c1, card_c2, card_c3, tiny_card, attenuated_card, batch_cards, CARDS)
from .draws import phantom, noise, random_vector

__all__ = ["Medium", "Grid", "Array", "Acquisition", "Prior", "PhantomSpec",
           "Card", "card_c1", "card_c2", "card_c3", "tiny_card", "attenuated_card", "batch_cards",
           "CARDS",
           "phantom", "noise", "random_vector"]
