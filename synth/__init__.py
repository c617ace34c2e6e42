"""Seeded synthetic inputs shared by the oracle, the tests and the bench."""
from .clouds import (Pair, config1, config2, config3, config4, config4_multistart, config5,
                     random_pair, rot_axis_angle, super_fibonacci_rotations)

__all__ = ["Pair", "config1", "config2", "config3", "config4", "config4_multistart", "config5",
           "random_pair", "rot_axis_angle", "super_fibonacci_rotations"]
