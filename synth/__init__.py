"""Seeded synthetic inputs: mechanisms and cell states.

Shared by the tests, the benchmark and the training-data driver.  Holds no
kinetics, integration or property arithmetic of the method itself."""
from .mechanism import Mechanism, generate, mech_small, mech_medium, mech_large, custom  # noqa: F401
