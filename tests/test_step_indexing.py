"""Index arithmetic of the multi-step forward kernels, modelled on the CPU.

The two- and three-step kernels (two or three stream-collide updates per pass
over HBM) hand intermediate populations between threads through LDS rings and
registers.  These tests restate the kernels' index formulas (block -> tile and
strip with the XCD-grouped order, thread -> column including the halo
columns, ring row of each plane and pass slot, register pipelines by c_y) and
check, for every block, thread and pass, what the kernels rely on:

* every LDS index is inside its array and no cell is written twice in a pass;
* every read of an update gets plane q of site (x - c_qx, y - c_qy) of the
  previous update's output, written in the pass the ring scheme says;
* every output site is written exactly once.

Read/write order within a pass follows the barriers (writes of an update
before the reads of the next one).  The tests do not run GPU code; the GPU
tests compare the kernels with single steps bit for bit.
"""
import pytest

# plane velocities in storage order (D2Q9, then the D2Q5 x and y components)
CX = (0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 1, 0, -1, 0, 0, 1, 0, -1, 0)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 1, 0, -1, 0, 0, 1, 0, -1)
# LDS group of the c_x != 0 planes (0: c_y = +1, 1: c_y = 0, 2: c_y = -1), -1 for c_x = 0
GROUP = (-1, 1, -1, 1, -1, 0, 0, 2, 2, -1, 1, -1, 1, -1, -1, 1, -1, 1, -1)
INDEX = (0, 0, 0, 1, 0, 0, 1, 0, 1, 0, 2, 0, 3, 0, 0, 4, 0, 5, 0)
NPLANES = {0: 2, 1: 6, 2: 2}
# a c_y = +1 plane is read two passes after it is written, c_y = 0 one, c_y = -1 the same
DELAY = {0: 2, 1: 1, 2: 0}
REG_DELAY = {1: 2, 0: 1, -1: 0}


def block_origin(b, tiles, strips, rows, width):
    if strips % 8 == 0:   # whole strips per XCD
        k = b >> 3
        strip, tile = (b & 7) + 8 * (k // tiles), k % tiles
    else:
        tile, strip = b % tiles, b // tiles
    return tile * width, strip * rows


def cmod(a, n):
    """C's remainder (the sign of the dividend), as the kernels compute it."""
    return -((-a) % n) if a < 0 else a % n


def gather_rows(r, ny):
    """t2_rows: the row r wrapped once and its two neighbours; all must lie
    in the lattice."""
    r = r + ny if r < 0 else (r - ny if r >= ny else r)
    rows = ((r + 1) if r < ny - 1 else 0, r, (r - 1) if r > 0 else ny - 1)
    assert all(0 <= v < ny for v in rows), (r, ny)
    return rows


def ring_row(q, t, slots):
    g = GROUP[q]
    base = {0: 0, 1: 2 * slots[0], 2: 2 * slots[0] + 6 * slots[1]}[g]
    return base + (t % slots[g]) * NPLANES[g] + INDEX[q]


def two_step(nx, ny, V, fp16):
    """k_step2: 256 threads of V sites, one halo column per side taken by
    threads 0 and 1, rings of 4 / 3 / 2 slots, one barrier per pass."""
    W = 256 * V
    tiles = (nx + W - 1) // W
    rows = max(8, min(32 if fp16 else 128, tiles * ny // (4096 if fp16 else 512)))
    strips = (ny + rows - 1) // rows
    slots = (4, 3, 2)
    nrows = 2 * 4 + 6 * 3 + 2 * 2
    written = set()
    for b in range(tiles * strips):
        x0, y0 = block_origin(b, tiles, strips, rows, W)
        wt, h = min(W, nx - x0), min(rows, ny - y0)
        lds, reg = {}, {}
        for t in range(h + 2):
            gather_rows(y0 - 1 + t, ny)
            r = (y0 - 1 + t) % ny
            sites = []
            for tid in range(256):
                if tid * V < wt:
                    sites += [(tid, j, x0 + tid * V + j, tid * V + j + 1, True) for j in range(V)]
                if tid < 2:
                    hx = ((x0 - 1) % nx) if tid == 0 else ((x0 + wt) % nx)
                    sites.append((tid, -1, hx, 0 if tid == 0 else wt + 1, False))
            cells = set()
            for tid, j, xc, col, own in sites:
                for q in range(19):
                    if GROUP[q] >= 0:
                        row = ring_row(q, t, slots)
                        assert 0 <= row < nrows and 0 <= col < W + 2
                        assert (row, col) not in cells
                        cells.add((row, col))
                        lds[(row, col)] = (q, xc, r, t)
                    elif own:
                        reg[(tid, j, q, t)] = (xc, r)
            if t < 2:
                continue
            r2 = y0 + t - 2
            for tid in range(256):
                for j in range(V):
                    lc = tid * V + j
                    if tid * V >= wt:
                        continue
                    x = x0 + lc
                    assert (x, r2) not in written
                    written.add((x, r2))
                    for q in range(19):
                        want = ((x - CX[q]) % nx, (r2 - CY[q]) % ny)
                        if GROUP[q] >= 0:
                            tt = t - DELAY[GROUP[q]]
                            got = lds[(ring_row(q, tt, slots), lc - CX[q] + 1)]
                            assert got == (q, *want, tt)
                            # the slot is not written again in the next pass
                            assert ring_row(q, t + 1, slots) != ring_row(q, tt, slots)
                        else:
                            assert reg[(tid, j, q, t - REG_DELAY[CY[q]])] == want
    assert len(written) == nx * ny


def t3_row(q):
    g, i = GROUP[q], INDEX[q]
    return i if g == 0 else (2 + i if g == 1 else 8 + i)


def three_step(nx, ny):
    """k_step_t3: 256 threads plus a fifth wave for the four halo columns,
    one LDS row per c_x != 0 plane and level, read by the consumer in the
    pass that writes it (right after the barrier) and carried on in its
    registers; two barriers per pass; the trajectory-storing variant writes
    each intermediate site once."""
    W, H = 256, 2
    tiles = (nx + W - 1) // W
    rows = tiles * ny // 512
    rows = 8 if rows < 8 else (32 if rows > 128 else rows)
    strips = (ny + rows - 1) // rows
    written = set()
    mids = [set(), set()]   # intermediate states stored by a trajectory-storing pass
    for b in range(tiles * strips):
        x0, y0 = block_origin(b, tiles, strips, rows, W)
        wt, h = min(W, nx - x0), min(rows, ny - y0)
        cols = []
        for tid in range(W + 64):
            if tid < W:
                cols.append((tid, tid < wt))
            else:
                k = tid - W
                cols.append(((-2, -1, wt, wt + 1)[k] if k < 4 else 0, k < 4))
        levels = [{}, {}]
        regs = [{}, {}]   # (thread, plane, pass) -> site whose level-s value the thread holds
        for t in range(h + 2 * H):
            for s in range(3):
                r = y0 - H + t - s
                if s == 0:
                    gather_rows(r, ny)
                if s > 0:
                    # every pass, each thread of the update's columns takes the
                    # c_x != 0 planes of the row just published at lc - c_x
                    for tid, (lc, has) in enumerate(cols):
                        if not (has and s - H <= lc <= wt - 1 + H - s):
                            continue
                        for q in range(19):
                            if GROUP[q] >= 0:
                                col = lc - CX[q] + H - (s - 1)
                                assert 0 <= col < W + 2 * (H - s + 1)
                                cell = levels[s - 1].get((t3_row(q), col))
                                if t >= 2 * (s - 1):
                                    assert cell is not None and cell[0] == q and cell[3] == t
                                    regs[s - 1][(tid, q, t)] = cell[1:3]
                cells = set()
                for tid, (lc, has) in enumerate(cols):
                    if not (has and t >= 2 * s and s - H <= lc <= wt - 1 + H - s):
                        continue
                    xc = (x0 + lc) % nx
                    if s > 0:
                        for q in range(19):
                            want = ((xc - CX[q]) % nx, (r - CY[q]) % ny)
                            assert regs[s - 1][(tid, q, t - REG_DELAY[CY[q]])] == want
                    if s < 2 and 0 <= lc < wt and 2 + s <= t <= h + 1 + s:
                        assert y0 <= r < y0 + h and (xc, r) not in mids[s]
                        mids[s].add((xc, r))
                    if s < 2:
                        for q in range(19):
                            if GROUP[q] >= 0:
                                key = (t3_row(q), lc + H - s)
                                assert 0 <= key[0] < 10 and 0 <= key[1] < W + 4 - 2 * s
                                assert key not in cells
                                cells.add(key)
                                levels[s][key] = (q, xc, r % ny, t)
                            else:
                                regs[s][(tid, q, t)] = (xc, r % ny)
                    else:
                        assert y0 <= r < y0 + h and 0 <= lc < wt
                        assert (xc, r) not in written
                        written.add((xc, r))
    assert len(written) == nx * ny
    assert len(mids[0]) == len(mids[1]) == nx * ny


def two_step_neighbours(nx, ny):
    """k_step_nb2: 256 threads plus a fifth wave for the six halo columns;
    pass t gathers row a = y0 - 3 + t (moments to ring m1), takes the first
    update of row a - 1 (gradients from m1, planes moving along x to one LDS
    row each), the second gather of row a - 2 (moments to ring m2) and the
    second update of row a - 3 (gradients from m2); three barriers per pass.
    Checks every moment read (site and pass), every population of both
    gathers, LDS bounds, single writes, and the trajectory-storing variant's
    intermediate sites."""
    W = 256
    tiles = (nx + W - 1) // W
    rows = tiles * ny // 512
    rows = 8 if rows < 8 else (32 if rows > 128 else rows)
    strips = (ny + rows - 1) // rows
    written, mids = set(), set()
    for b in range(tiles * strips):
        x0, y0 = block_origin(b, tiles, strips, rows, W)
        wt, h = min(W, nx - x0), min(rows, ny - y0)
        cols = []
        for tid in range(W + 64):
            if tid < W:
                cols.append((tid, tid < wt))
            else:
                k = tid - W
                cols.append(((k - 3 if k < 3 else wt + k - 3) if k < 6 else 0, k < 6))
        m1, m2, y1 = {}, {}, {}
        p1c, p2c = {}, {}            # tid -> site whose gather the thread holds from the last pass
        zc, zu1, zu2 = {}, {}, {}    # tid -> {q: site} of the c_x = 0 first-update planes
        xc1, xu1, xu2 = {}, {}, {}   # tid -> {q: site} of the carried c_x != 0 planes
        for t in range(h + 6):
            a = y0 - 3 + t
            aw = cmod(a, ny)
            gather_rows(aw + ny if aw < 0 else aw, ny)
            s0, s1, s2 = t % 3, (t - 1) % 3, (t - 2) % 3
            site = {}
            # 1. gather row a, moments to m1 at column lc + 3
            cells = set()
            p1n = {}
            for tid, (lc, has) in enumerate(cols):
                if not has:
                    continue
                xc = (x0 + lc) % nx
                site[tid] = xc
                key = (s0, lc + 3)
                assert 0 <= key[1] < W + 6 and key not in cells
                cells.add(key)
                m1[key] = ((xc, a % ny), t)
                p1n[tid] = (xc, a % ny)
            # 2. first update of row a - 1
            cells, n2 = set(), {}
            for tid, (lc, has) in enumerate(cols):
                if not (has and -2 <= lc <= wt + 1 and t >= 2):
                    continue
                xc = site[tid]
                r = a - 1
                for dy, sl in ((-1, s2), (0, s1), (1, s0)):
                    for dx in (-1, 0, 1):
                        c = lc + 3 + dx
                        assert 0 <= c < W + 6
                        assert m1[(sl, c)] == (((xc + dx) % nx, (r + dy) % ny), t + dy - 1)
                assert p1c[tid] == (xc, r % ny)
                if 0 <= lc < wt and y0 <= r < y0 + h:
                    assert (xc, r) not in mids
                    mids.add((xc, r))
                n2[tid] = {}
                for q in range(19):
                    if GROUP[q] >= 0:
                        key = (t3_row(q), lc + 2)
                        assert 0 <= key[1] < W + 4 and key not in cells
                        cells.add(key)
                        y1[key] = (q, xc, r % ny, t)
                    else:
                        n2[tid][q] = (xc, r % ny)
            # 3. second gather of row a - 2: every thread takes the y1 values of
            # this pass at lc + 2 - c_x (threads without the gather at 2 - c_x)
            cells, p2n = set(), {}
            for tid, (lc, has) in enumerate(cols):
                up3 = has and -1 <= lc <= wt
                c3 = lc + 2 if up3 else 2
                e = {}
                for q in range(19):
                    if GROUP[q] >= 0:
                        col = c3 - CX[q]
                        assert 0 <= col < W + 4
                        e[q] = y1.get((t3_row(q), col))
                if up3 and t >= 4:
                    xc, r = site[tid], a - 2
                    for q in range(19):
                        want = ((xc - CX[q]) % nx, (r - CY[q]) % ny)
                        if GROUP[q] >= 0:
                            got = {1: xu2, 0: xc1, -1: {tid: e}}[CY[q]][tid][q]
                            assert got is not None and got[0] == q and got[1:3] == want
                            assert got[3] == t - REG_DELAY[CY[q]]
                        else:
                            got = {0: zc, 1: zu2, -1: n2}[CY[q]][tid][q]
                            assert got == want
                    key = (s0, lc + 1)
                    assert 0 <= key[1] < W + 2 and key not in cells
                    cells.add(key)
                    m2[key] = ((xc, r % ny), t)
                    p2n[tid] = (xc, r % ny)
                xu2[tid] = {q: v for q, v in xu1.get(tid, {}).items()}
                xu1[tid] = {q: v for q, v in e.items() if CY[q] == 1}
                xc1[tid] = {q: v for q, v in e.items() if CY[q] == 0}
            # 4. second update of row a - 3, stored
            for tid, (lc, has) in enumerate(cols):
                if not (has and 0 <= lc < wt and t >= 6):
                    continue
                xc, r = site[tid], a - 3
                for dy, sl in ((-1, s2), (0, s1), (1, s0)):
                    for dx in (-1, 0, 1):
                        c = lc + 1 + dx
                        assert 0 <= c < W + 2
                        assert m2[(sl, c)] == (((xc + dx) % nx, (r + dy) % ny), t + dy - 1)
                assert p2c[tid] == (xc, r % ny)
                assert y0 <= r < y0 + h and (xc, r) not in written
                written.add((xc, r))
            for tid, (lc, has) in enumerate(cols):
                p1c[tid] = p1n.get(tid)
                p2c[tid] = p2n.get(tid)
                zu2[tid] = zu1.get(tid, {})
                zu1[tid] = {q: v for q, v in n2.get(tid, {}).items() if CY[q] == 1}
                zc[tid] = {q: v for q, v in n2.get(tid, {}).items() if CY[q] == 0}
    assert len(written) == nx * ny
    assert len(mids) == nx * ny


SIZES = [(256, 64), (300, 70), (2, 2), (3, 5), (513, 9), (600, 60), (77, 41), (4, 600)]


@pytest.mark.parametrize("nx,ny", SIZES)
def test_two_step_fp32_index_model(nx, ny):
    two_step(nx, ny, 1, False)


@pytest.mark.parametrize("nx,ny", [(512, 40), (600, 70), (2, 2), (1030, 124), (600, 34)])
def test_two_step_fp16_pairs_index_model(nx, ny):
    two_step(nx, ny, 2, True)


@pytest.mark.parametrize("nx,ny", [(301, 33), (3, 3), (77, 41)])
def test_two_step_fp16_odd_index_model(nx, ny):
    two_step(nx, ny, 1, True)


@pytest.mark.parametrize("nx,ny", SIZES + [(5, 3)])
def test_three_step_index_model(nx, ny):
    three_step(nx, ny)


@pytest.mark.parametrize("nx,ny", SIZES + [(5, 3), (258, 17), (2, 3)])
def test_two_step_neighbour_closures_index_model(nx, ny):
    two_step_neighbours(nx, ny)


@pytest.mark.parametrize("tiles,strips", [(1, 8), (3, 8), (16, 32), (5, 64), (32, 64)])
def test_xcd_order_is_a_bijection(tiles, strips):
    seen = {block_origin(b, tiles, strips, 1, 1) for b in range(tiles * strips)}
    assert seen == {(x, y) for x in range(tiles) for y in range(strips)}
