"""Seeded synthetic inputs for the encrypted-GCN workloads.

This package only draws random graphs, features and weights with numpy's
PCG64 generator.  It holds none of the method's arithmetic (no normalisation,
no encoding, no modular arithmetic), so both the CPU oracle and the GPU
library can take their inputs from it without sharing any computation.
"""
from .graphs import (Graph, erdos_renyi, chung_lu, dc_sbm, sample_neighbors)
from .features import (binary_features, uniform_features, tfidf_features,
                       gaussian_weights)
from .configs import CONFIGS, make_workload, Workload
from .ciphertexts import uniform_ct_words

__all__ = ["Graph", "erdos_renyi", "chung_lu", "dc_sbm", "sample_neighbors",
           "binary_features", "uniform_features", "tfidf_features",
           "gaussian_weights", "CONFIGS", "make_workload", "Workload", "uniform_ct_words"]
