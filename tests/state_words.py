"""Stored words of an encoded lattice (test helper).

A lattice holds 19 planes of ny rows, each row padded to a pitch of whole
256-byte blocks; the kernels never read or write the padding, so it holds
whatever the buffer held before.  Bitwise comparisons of states therefore take
the stored elements only: int32 words for FP32 storage, int16 for FP16.
"""
import torch


def stored_words(lat, state: torch.Tensor | None = None) -> torch.Tensor:
    """(19, ny, nx) view of the stored words of `state` (default: the current
    state of lattice `lat`), on the device."""
    c = lat.cfg
    es = 4 if c.storage == "fp32" else 2
    pitch = lat.lattice_bytes // (19 * c.ny * es)
    dt = torch.int32 if es == 4 else torch.int16
    st = lat.save_state() if state is None else state
    return st[: lat.lattice_bytes].view(dt).view(19, c.ny, pitch)[:, :, : c.nx]
