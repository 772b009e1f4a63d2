"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .field import FieldRecipe, field_digest, make_field, plane_wave_field, power_amplitude

__all__ = ["FieldRecipe", "make_field", "field_digest", "plane_wave_field", "power_amplitude"]
