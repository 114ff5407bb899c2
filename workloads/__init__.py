"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

Holds circuit construction, a statevector simulator standing in for the
quantum processors, wire cutting into measured subcircuit variants, and
synthetic Pauli-basis tensors.  None of the reconstruction arithmetic lives
here.
"""
from .circuit import Circuit, Gate, statevector, probabilities  # noqa: F401
from .cutting import Network, TensorSpec, cut_circuit  # noqa: F401
