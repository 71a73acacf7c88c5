"""Memory sizes of materialised intermediates (test infrastructure only).

The paper sizes the attention logits of the fine-tuning extra-MSA row
attention (Section "Subbatch VS DAP", the logits equation): N_seq * N_head *
N_res^2 elements of BFloat16, 11.25 GiB at [5120, 8, 384], and 1.125 GiB once
the MSA rows are processed in chunks of 512.  Its Subbatch figure sizes a
[rows, cols] BFloat16 activation the same way (20 bytes for [2, 5], 10 bytes
with chunk 1).
"""
from __future__ import annotations


def logits_bytes(n_seq: int, n_head: int, n_res: int, elem_bytes: int = 2, chunk: int = 0) -> int:
    """Bytes of one materialised [rows, N_head, N_res, N_res] logits tensor,
    rows = N_seq, or ``chunk`` rows at a time when chunked."""
    rows = n_seq if chunk <= 0 else min(chunk, n_seq)
    return rows * n_head * n_res * n_res * elem_bytes


def activation_bytes(rows: int, cols: int, elem_bytes: int = 2, chunk: int = 0) -> int:
    """Peak bytes of a [rows, cols] intermediate when ``chunk`` rows are live."""
    live = rows if chunk <= 0 else min(chunk, rows)
    return live * cols * elem_bytes
