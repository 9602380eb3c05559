"""Seeded synthetic inputs for the ray-shooting path.

This package is the ONE piece shared by the HIP path's callers and the oracle:
it draws random numbers and turns them into lens arrays and workload
descriptions.  It holds none of the method's arithmetic (no deflection, no
geometry rules, no binning): the lens rectangle and the lens count are passed
in by the caller, who gets them from whichever side it is exercising.
"""
from .rng import splitmix64, uniform01
from .lenses import Lenses, uniform_lenses, disc_lenses, salpeter_mean_mass
from . import configs
from . import network

__all__ = ["splitmix64", "uniform01", "Lenses", "uniform_lenses", "disc_lenses",
           "salpeter_mean_mass", "configs", "network"]
