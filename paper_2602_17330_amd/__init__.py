"""SubQuad hot path on AMD Instinct MI355X (gfx950): MinHash -> LSH candidates ->
Smith-Waterman -> gated fusion (forward and backward), behind the C ABI of
``include/subquad.h`` (libsubquad.so). The Python layer only marshals arguments."""
from ._lib import LIB_PATH, SIGNATURES, SubquadError, lib  # noqa: F401
from .api import (GateFn, align, align_nows, check_seqs, check_subst, edit_cost_matrix,  # noqa: F401
                  edit_distance, gate3_bwd, gate3_fwd, gate_bwd,
                  gate_fwd, graph_topk, lsh_candidates, minhash, self_scores, to_device)
