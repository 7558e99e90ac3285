"""MI355X-native three-phase leaky-dielectric EHD lattice Boltzmann step.

The compute path is the HIP library ``liblbm_ehd.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/lbm_ehd.h``; ``binding`` marshals
arguments to it.  ``inputs`` builds seeded synthetic workloads.  Importing the
package loads nothing; ``binding`` loads the library on first use and raises
if it is missing.
"""
__all__ = ["binding", "inputs"]
