"""Seeded synthetic inputs shared by the product path and the oracle.

Nothing here contracts or plans: circuits, gate matrices and the labelled-leg
networks built from them.
"""
from .circuits import (Circuit, Gate, gate_matrix, ghz, hadamard_layer, phase_poly_circuit,
                       graph_state_circuit, brick_edges,
                       brickwork_circuit, random_circuit, random_bitstrings, circuit_mix,
                       zipf_indices)
from .network import (Network, amplitude_network, amplitude_overrides, output_tensor_ids,
                      zz_network, lightcone, basis_vec)
