"""Memory-sized batching of repertoires (Eq. (batch), "Data normalization and hardware-aware
batching").

The paper sizes a batch as B = min(|S|, max(32, floor(sqrt(M_avail / (c * l_max))))): the
square root belongs to an all-pairs B x B comparison tile.  Behind the MinHash prefilter the
footprint of a batch grows linearly in its sequences (signatures, band records, embeddings
and the candidate pairs each sequence brings), so the batch planner below uses the same
rule with that linear footprint: whole repertoires are packed, in order, into batches whose
estimated bytes stay within the device memory available.
"""
from __future__ import annotations

import math


def eq_batch(n_avail: int, mem_avail: float, c: float, l_max: int) -> int:
    """Eq. (batch) as printed (all-pairs tile of B x B sequences)."""
    return int(min(n_avail, max(32, math.floor(math.sqrt(mem_avail / (c * l_max))))))


def bytes_per_sequence(M: int, b: int, d: int, stride: int, pairs_per_seq: float) -> float:
    """Device bytes one sequence brings to a batch on the hot path."""
    per_seq = (stride + 4 + 4 + 4 + 4          # sequence row, length, V-gene, family, self-score
               + 8 * M                          # signature row
               + 2 * 8 * b                      # band records (two sort buffers)
               + 4 * ((b + 3) // 4 * 4)         # exact class ids, rows padded to 16 bytes
               + 8 + 16                         # CSR row offset, gate node record
               + 2 * 4 * d)                     # embedding and its gradient
    per_pair = (8 + 2 * 8                        # pair, pair-sort keys (x2)
                + 4 + 4 + 4                      # score, fused, upstream gradient
                + 2 * 8 + 16                     # alignment length sort (x2), metadata record
                + 4 * 8 + 16 + 16)               # gate pair orders (x4), per-pair records (2 x 16)
    return per_seq + pairs_per_seq * per_pair


def plan_batches(sizes, bytes_per_seq: float, mem_avail: float, headroom: float = 0.85) -> list[list[int]]:
    """Pack whole repertoires (in order) into batches that fit ``headroom * mem_avail``."""
    budget = headroom * mem_avail
    batches, cur, cur_bytes = [], [], 0.0
    for r, n in enumerate(sizes):
        need = n * float(bytes_per_seq)
        if cur and cur_bytes + need > budget:
            batches.append(cur)
            cur, cur_bytes = [], 0.0
        cur.append(r)
        cur_bytes += need
    if cur:
        batches.append(cur)
    return batches
