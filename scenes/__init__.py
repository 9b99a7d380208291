"""Seeded synthetic bundle-adjustment scenes (inputs only; no solver arithmetic)."""
from .generate import Scene, make_scene, SCENE_NAMES, subscene

__all__ = ["Scene", "make_scene", "SCENE_NAMES", "subscene"]
