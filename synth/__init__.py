"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

Holds only random draws and configuration numbers (box sizes, counts,
parameter values); none of the model's arithmetic lives here.
"""
from .configs import *  # noqa: F401,F403
