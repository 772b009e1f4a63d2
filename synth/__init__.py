"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .field import FieldRecipe, field_digest, make_field, plane_wave_field, power_amplitude

__all__ = ["FieldRecipe", "make_field", "field_digest", "plane_wave_field", "power_amplitude", "make_field_torch"]


def make_field_torch(*args, **kwargs):
    """See synth.field_torch (imported lazily so numpy-only users need no torch)."""
    from .field_torch import make_field_torch as _impl

    return _impl(*args, **kwargs)
