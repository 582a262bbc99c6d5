"""The encoded layout (GPU): lbmhd_layout's row pitch and plane stride.

Population q of site (x, y) is element q * plane + y * pitch + x of a state
(q * adj_plane + y * adj_pitch + x of an adjoint lattice); rows are padded to
whole 256-byte blocks and successive planes are spaced by a further 768-byte
gap.  The tests check that the stored elements sit where the layout says (the
FP16 encoding of known populations read back through it), and that no kernel
writes the row padding or the gaps: both bound lattices, the stored
trajectories and the adjoint buffers are filled with a sentinel byte first,
then every kind of pass runs (one, two and three steps per pass, in place,
the closures that read the neighbours, the stored trajectories, single and
paired reverse steps, the kinetic closure's reverse step), and every byte
outside the stored elements must still hold the sentinel.  Lattices 300 x 70
(FP32 rows padded from 1200 to 1280 bytes) and 100 x 36 (FP16: 200 to 256
bytes).
"""
import numpy as np
import pytest
import torch

from lbmhd_inputs import orszag_tang

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def element_mask(nbytes, plane, pitch, nx, ny, esize, nplanes=19):
    """Boolean (nbytes,) mask of the bytes that hold stored elements."""
    m = torch.zeros(nbytes // esize, dtype=torch.bool)
    q = torch.arange(nplanes)[:, None, None]
    y = torch.arange(ny)[None, :, None]
    x = torch.arange(nx)[None, None, :]
    m[(q * plane + y * pitch + x).reshape(-1)] = True
    return m.repeat_interleave(esize)


def untouched(buf, mask):
    """The bytes of buf outside mask still hold the sentinel."""
    other = buf.cpu()[: mask.numel()][~mask]
    return bool((other == SENTINEL).all()), int((other != SENTINEL).sum())


def test_layout_places_every_population(lb):
    nx, ny = 100, 36
    L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny, storage="fp16"))
    assert (L.pitch, L.plane) == (128, 36 * 128 + 384)
    assert (L.adj_pitch, L.adj_plane) == (128, 36 * 128 + 192)
    assert L.lattice_bytes == 19 * L.plane * 2 and L.adj_lattice_bytes == 19 * L.adj_plane * 4
    w9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    w19 = np.concatenate([w9, np.zeros(10)])
    q, y, x = np.meshgrid(np.arange(19), np.arange(ny), np.arange(nx), indexing="ij")
    pops = w19[:, None, None] + 1e-4 * ((q * 7 + y * 3 + x) % 23 - 11)
    L.set_populations(pops)
    raw = L.save_state().view(torch.float16).cpu()
    # the encoding: half(2^10 * float(f - w)), rounded to nearest even
    dev = (pops - w19[:, None, None]).astype(np.float32)
    want = torch.from_numpy((np.float32(1024) * dev).astype(np.float16))
    got = raw[torch.from_numpy((q * L.plane + y * L.pitch + x).reshape(-1))].reshape(19, ny, nx)
    assert torch.equal(got.view(torch.int16), want.view(torch.int16))
    assert torch.equal(L.state_view().cpu().view(torch.int16), want.view(torch.int16))


@pytest.mark.parametrize("storage,nx,ny", [("fp32", 300, 70), ("fp16", 100, 36)])
@pytest.mark.parametrize("kind", ["single", "pairs", "triples", "inplace", "kinetic",
                                  "cross-helicity", "store", "adjoint", "kinetic-adjoint"])
def test_no_kernel_writes_padding_or_gaps(lb, storage, nx, ny, kind):
    print(f"\nlayout {kind} {storage} {nx}x{ny}", flush=True)
    esize = 4 if storage == "fp32" else 2
    les = {"kinetic": 2, "cross-helicity": 4, "kinetic-adjoint": 3}.get(kind, 1)
    spp = {"single": 1, "pairs": 2, "triples": 3}.get(kind, 0)
    if kind in ("kinetic", "cross-helicity"):
        spp = 2
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-3, eta=2e-3, les=les, cs=0.1, delta=1.0,
                         storage=storage, steps_per_pass=spp, inplace=kind == "inplace")
    L = lb.Lattice(cfg)
    bufs = [t for t in (L._a, L._b) if t is not None]
    for t in bufs:
        t.fill_(SENTINEL)
    mask = element_mask(L.lattice_bytes, L.plane, L.pitch, nx, ny, esize)
    L.init_fields(*orszag_tang(nx, ny))
    extra = []
    if kind == "store":
        store = torch.full((5, L.lattice_bytes), SENTINEL, dtype=torch.uint8, device="cuda")
        L.step_store(L.save_state(), store, 5)
        half = torch.full((2, L.lattice_bytes), SENTINEL, dtype=torch.uint8, device="cuda")
        L.step_store_pairs(L.save_state(), half, 2)
        extra = [store[i] for i in range(5)] + [half[i] for i in range(2)]
    elif kind in ("adjoint", "kinetic-adjoint"):
        amask = element_mask(L.adj_lattice_bytes, L.adj_plane, L.adj_pitch, nx, ny, 4)
        x0 = L.save_state()
        lam = [L.new_adj_buffer() for _ in range(3)]
        for t in lam:
            t.view(torch.uint8).fill_(SENTINEL)
        acc = L.new_adj_acc()
        L.adj_seed_energy(x0, lam[0])
        L.adj_step(x0, lam[0], lam[1], acc)
        if kind == "adjoint":
            L.adj_step2(x0, lam[1], lam[2], acc)
        else:
            L.adj_step(x0, lam[1], lam[2], acc)
        torch.cuda.synchronize()
        for t in lam:
            ok, bad = untouched(t.view(torch.uint8), amask)
            assert ok, bad
    else:
        L.step(7)
    L.diag()
    torch.cuda.synchronize()
    for t in bufs + extra:
        ok, bad = untouched(t, mask)
        assert ok, bad
    assert L.diag()["nonfinite"] == 0
