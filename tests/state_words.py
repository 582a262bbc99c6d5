"""Stored words of an encoded lattice (test helper).

A lattice holds 19 planes of ny rows, each row padded to a pitch of whole
256-byte blocks and successive planes spaced by a further gap
(lbmhd_layout); the kernels never read or write the padding or the gaps, so
they hold whatever the buffer held before.  Bitwise comparisons of states
therefore take the stored elements only: int32 words for FP32 storage, int16
for FP16.
"""
import torch


def stored_words(lat, state: torch.Tensor | None = None) -> torch.Tensor:
    """(19, ny, nx) view of the stored words of `state` (default: the current
    state of lattice `lat`), on the device."""
    c = lat.cfg
    dt = torch.int32 if c.storage == "fp32" else torch.int16
    st = lat.save_state() if state is None else state
    return st[: lat.lattice_bytes].view(dt).as_strided((19, c.ny, c.nx), (lat.plane, lat.pitch, 1))
