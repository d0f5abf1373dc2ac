"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This package only *draws* inputs (gate lists, sampled basis indices, request
traces). It applies no gate and holds none of the simulator's arithmetic, so
the oracle and the device path can both consume its output without sharing any
of the method's code.
"""

from .circuits import (  # noqa: F401
    GATE_DTYPE, KIND_U, KIND_CX, KIND_CZ, KIND_CU,
    H, X, Y, Z, phase,
    haar_u2, layered_circuit, paper_random_circuit, qft_like_circuit,
    qft_circuit, ghz_circuit, sample_indices, mixed_circuit, make_gates,
    config_circuit, config_samples, batch_workload, request_trace,
    CONFIGS, MASTER_SEED,
)
