"""Seeded synthetic multicommodity-flow instances (inputs only; no PDR arithmetic)."""
from .instance import Instance, load_instance, recipe_small, RECIPES, stream  # noqa: F401
