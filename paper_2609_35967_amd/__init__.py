"""MI355X (gfx950) library for the collision hot path of the GameDev
representative-particle dust model (arXiv 2609.35967): exact kNN on a Morton
LBVH, frozen-neighbourhood pair rates and interval plan, Philox-driven Monte
Carlo sampling, and the staggered semi-analytic push, behind the C ABI of
include/gd.h.  ``binding`` marshals arguments; all compute is in libgd.so.
"""
from .binding import Engine, GdError, load, make_problem  # noqa: F401

__all__ = ["Engine", "GdError", "load", "make_problem"]
