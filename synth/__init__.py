"""Seeded synthetic inputs for the SubQuad hot path.

This package is the only code shared by the CPU oracle and the GPU path. It produces
inputs (sequences, lengths, family/V-gene/subgroup labels, embeddings, gate weights, pair
lists, the substitution matrix) and holds none of the method's arithmetic.
"""
from .alphabet import ALPHABET, PAD, decode, encode, load_blosum62  # noqa: F401
from .inputs import (embeddings, gate_params, random_pairs, sample_rows,  # noqa: F401
                     upstream_grad)
from .repertoire import (HASH_SEED, GATE_HIDDEN, WORKLOADS, Repertoire,  # noqa: F401
                         batch64, batch_sizes, concat, rep1m, small5k, tiny,
                         zipf100k, zipf_rank_sizes)
