"""MI355X-native per-cell radiation-hydrodynamics update of QUOKKA
(Wibking & Krumholz 2021, arXiv:2110.01792).

The compute path is the HIP library built from csrc/ (libquokka_mi355x.so,
C ABI declared in include/quokka.h); `binding` marshals arguments to it.
`inputs` holds the seeded synthetic workloads.  Importing the package loads
nothing; the binding loads the library on first use and raises if it is
missing.
"""
__all__ = ["binding", "inputs"]
