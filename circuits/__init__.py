"""Seeded synthetic circuit and bitstring generators.

This package holds inputs only: gate matrices under fixed conventions, lattice
layouts, the random circuit families the workloads are drawn from, and the
output bitstrings.  It contains none of the contraction arithmetic; both the
CPU oracle and the GPU path read the same circuit object (gate list with
complex128 matrices) and build their own tensor networks from it.

Conventions (written out in CONVENTIONS.md beside this file):
  * qubit q on an R x C lattice is q = r*C + c; on an X x Y x Z stack it is
    q = x + X*y + X*Y*z;
  * a two-qubit matrix is indexed row = 2*o(q1) + o(q2), column likewise for
    the inputs, with q1 the first listed qubit;
  * bit q of a packed uint64 bitstring is the output value of qubit q;
  * the initial state is |0...0>.
"""
from .gates import (H, SQRT_X, SQRT_Y, SQRT_W, CZ, z_phase, cphase, fsim,
                    haar_su2, haar_su4)
from .model import Circuit, Gate
from .families import (lattice_circuit, iqp_lattice_circuit, stack3d_circuit,
                       product_circuit, mirror, make_config, config_names,
                       random_bitstrings, pack_bits, unpack_bits,
                       circuit_seed, bitstring_seed, paper_iqp_circuit,
                       sycamore_type_circuit, paper_family_instances,
                       sycamore_type_gate_counts, cavity_circuit_gate_counts,
                       cavity_circuit)

__all__ = [
    "H", "SQRT_X", "SQRT_Y", "SQRT_W", "CZ", "z_phase", "cphase", "fsim",
    "haar_su2", "haar_su4", "Circuit", "Gate", "lattice_circuit",
    "iqp_lattice_circuit", "stack3d_circuit", "product_circuit", "mirror",
    "make_config", "config_names", "random_bitstrings", "pack_bits",
    "unpack_bits", "circuit_seed", "bitstring_seed", "paper_iqp_circuit",
    "sycamore_type_circuit", "paper_family_instances", "sycamore_type_gate_counts",
    "cavity_circuit_gate_counts", "cavity_circuit",
]
