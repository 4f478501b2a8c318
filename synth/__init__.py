"""Seeded synthetic inputs (scenes, rigs, raw captures) shared by the tests, the
benchmark and the oracle checks.  Forward image model only: no reconstruction
arithmetic lives here."""
from . import configs, rig, scene  # noqa: F401
