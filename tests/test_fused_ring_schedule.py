"""Host-side replay of the fused two-step pass's data flow (the D3Q19 tiles
walking z and the D2Q9 segments walking y).

The fused pass collides the first step of each plane (row) on its tile and a
one-site halo, pushes the post-collision populations that land inside the
tile into a ring of LDS slots, and collides the second step of the plane two
phases later from that ring, with one barrier per phase.  This replays, with
plain integers and the identity collision, what the kernels do: the tile and
chunk decomposition with ragged and wrapping tiles, the first-step sites of
the interior, halo-row and halo-column waves, the ring (one flat array in the
kernels' LDS layout, so a push outside the tile corrupts a neighbouring row)
and the slots each phase writes and reads, and the second step's push into
the destination, and checks that:
  - one pass moves every population by 2 c_i (two steps of Eq. LBE's
    streaming, periodic), which fails if a slot were read before its plane
    is complete or overwritten before it is read;
  - within a phase the first step's slots and the second step's slots are
    disjoint, so one barrier per phase suffices;
  - the halo-column wave's lanes cover the rows -1 .. TH of the tile;
  - the slice descriptors of lattices with planes of 4 GiB or more (one
    z-plane or row per descriptor) reach every site's byte address with a
    lane offset inside the descriptor's 32-bit range.
It needs no GPU; the GPU tests check the compiled kernels bit for bit
against single steps and against the oracle."""
import numpy as np
import pytest

import oracle

C3 = oracle.tables(oracle.D3Q19)[0]
C2 = oracle.tables(oracle.D2Q9)[0]


def slots_written(it):
    """(flat, up, down) slots the first step of phase it writes."""
    return (it + 2) % 3, it % 4, it & 1


def slots_read(it):
    """(flat, up, down) slots the second step of phase it reads."""
    return it % 3, (it + 1) % 4, (it + 1) & 1


def cls(c):
    """Ring class of a population by its component along the walking axis."""
    return 0 if c == 0 else (1 if c > 0 else 2)


class Ring:
    """The LDS ring as one flat array in the kernels' layout: for each class
    (flat, up-going, down-going) its slots (3, 4, 2), each holding the
    class's populations (in population order) as planes of TP values."""
    SLOTS = (3, 4, 2)

    def __init__(self, walk, TP):
        self.TP = TP
        self.cls = [cls(c) for c in walk]
        self.idx = [sum(1 for j in range(i) if self.cls[j] == self.cls[i]) for i in range(len(walk))]
        n = [self.cls.count(k) for k in range(3)]
        self.base = [0, self.SLOTS[0] * n[0] * TP, self.SLOTS[0] * n[0] * TP + self.SLOTS[1] * n[1] * TP]
        self.n = n
        self.data = np.full(self.base[2] + self.SLOTS[2] * n[2] * TP, np.nan)

    def at(self, i, slots, pos):
        k = self.cls[i]
        return self.base[k] + slots[k] * self.n[k] * self.TP + self.idx[i] * self.TP + pos


def fused_pass_3d(state, TX, TY, ZLEN):
    """One fused pass with the identity collision over a D3Q19 state
    (19, nz, ny, nx) in the even layout; returns the state two steps later."""
    q, nz, ny, nx = state.shape
    out = np.full_like(state, np.nan)
    for z0 in range(0, nz, ZLEN):
        ZC = min(ZLEN, nz - z0)
        for y0 in range(0, ny, TY):
            TH = min(TY, ny - y0)
            for x0 in range(0, nx, TX):
                TW = min(TX, nx - x0)
                ring = Ring(C3[:, 2], TX * TY)
                # first-step sites of the waves: interior rows, the two halo
                # rows, and the halo-column wave (lanes h = 0..31 per side: rows h - 1)
                sites = [(sx, sy) for sy in range(TH) for sx in range(TW)]
                sites += [(sx, sy) for sy in (-1, TH) for sx in range(TW)]
                sites += [(sx, h - 1) for sx in (-1, TW) for h in range(32) if h < TH + 2]
                assert len(set(sites)) == len(sites) == (TW + 2) * (TH + 2)
                for it in range(ZC + 3):
                    w_slots = slots_written(it)
                    r_slots = slots_read(it)
                    assert all(w != r for w, r in zip(w_slots, r_slots)), it
                    if it <= ZC + 1:
                        u = (z0 + it - 1) % nz
                        for sx, sy in sites:
                            gx, gy = (x0 + sx) % nx, (y0 + sy) % ny
                            for i in range(q):
                                tx, ty = sx + C3[i, 0], sy + C3[i, 1]
                                if 0 <= tx < TW and 0 <= ty < TH:
                                    ring.data[ring.at(i, w_slots, ty * TX + tx)] = state[i, u, gy, gx]
                    if it >= 3:
                        z = z0 + it - 3
                        for ty in range(TH):
                            for tx in range(TW):
                                x, y = x0 + tx, y0 + ty
                                for i in range(q):
                                    v = ring.data[ring.at(i, r_slots, ty * TX + tx)]
                                    out[i, (z + C3[i, 2]) % nz, (y + C3[i, 1]) % ny, (x + C3[i, 0]) % nx] = v
    return out


def fused_pass_2d(state, SW, YLEN, NW):
    """One fused pass with the identity collision over a D2Q9 state
    (9, 1, ny, nx): segments of SW sites, NW segment waves (lanes w * 64 + l)
    and the halo-column wave (lanes 0 and 1)."""
    q, _, ny, nx = state.shape
    out = np.full_like(state, np.nan)
    for y0 in range(0, ny, YLEN):
        YC = min(YLEN, ny - y0)
        for x0 in range(0, nx, SW):
            TW = min(SW, nx - x0)
            ring = Ring(C2[:, 1], SW)
            sites = [w * 64 + l for w in range(NW) for l in range(64) if w * 64 + l < TW] + [-1, TW]
            for it in range(YC + 3):
                w_slots, r_slots = slots_written(it), slots_read(it)
                assert all(w != r for w, r in zip(w_slots, r_slots)), it
                if it <= YC + 1:
                    u = (y0 + it - 1) % ny
                    for sx in sites:
                        gx = (x0 + sx) % nx
                        for i in range(q):
                            tx = sx + C2[i, 0]
                            if 0 <= tx < TW:
                                ring.data[ring.at(i, w_slots, tx)] = state[i, 0, u, gx]
                if it >= 3:
                    y = y0 + it - 3
                    for tx in range(TW):
                        x = x0 + tx
                        for i in range(q):
                            v = ring.data[ring.at(i, r_slots, tx)]
                            out[i, 0, (y + C2[i, 1]) % ny, (x + C2[i, 0]) % nx] = v
    return out


@pytest.mark.parametrize("dims,tile", [((5, 3, 2), (64, 10, 32)), ((1, 1, 1), (64, 10, 32)),
                                       ((2, 2, 2), (64, 10, 32)), ((70, 13, 9), (64, 10, 4)),
                                       ((3, 29, 7), (64, 10, 3)), ((9, 4, 5), (4, 3, 1)),
                                       ((66, 21, 6), (64, 10, 32))])
def test_fused_pass_3d_streams_twice(dims, tile):
    nx, ny, nz = dims
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    state = rng.standard_normal((19, nz, ny, nx))
    out = fused_pass_3d(state, *tile)
    for i in range(19):
        want = np.roll(state[i], shift=(2 * C3[i, 2], 2 * C3[i, 1], 2 * C3[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(out[i], want), (dims, tile, i)


@pytest.mark.parametrize("dims,seg", [((5, 3), (256, 32, 4)), ((1, 1), (256, 32, 4)), ((2, 2), (256, 32, 4)),
                                      ((300, 7), (256, 32, 4)), ((257, 70), (256, 32, 4)),
                                      ((9, 11), (4, 3, 1)), ((130, 5), (64, 2, 1))])
def test_fused_pass_2d_streams_twice(dims, seg):
    nx, ny = dims
    rng = np.random.default_rng(nx * 100 + ny)
    state = rng.standard_normal((9, 1, ny, nx))
    out = fused_pass_2d(state, *seg)
    for i in range(9):
        want = np.roll(state[i], shift=(2 * C2[i, 1], 2 * C2[i, 0]), axis=(1, 2))
        assert np.array_equal(out[i], want), (dims, seg, i)


def test_ring_slot_lifetimes():
    """Each (class, slot) written for a plane is read by that plane's second
    step before the first step writes it again (for chunks of 1 to 40
    planes): the flat class is written one phase before it is read, the
    up-going class three phases before, the down-going class one phase
    before, and each is rewritten only after its read."""
    for ZC in range(1, 41):
        holder = {}
        for it in range(ZC + 3):
            ws, rs = slots_written(it), slots_read(it)
            if it >= 3:
                v = it - 3
                for k in range(3):
                    assert holder.get((k, rs[k])) == v, (ZC, it, k)
                    holder[(k, rs[k])] = "read"
            if it <= ZC + 1:
                u = it - 1
                for k, target in enumerate((u, u + 1, u - 1)):
                    prev = holder.get((k, ws[k]))
                    # a slot may be overwritten if it was read, never filled, or
                    # held a plane outside the chunk (never read)
                    assert prev in (None, "read") or not (0 <= prev < ZC), (ZC, it, k, prev)
                    holder[(k, ws[k])] = target


def _slice_access(base, plane_elems, plane, slice_idx, slice_elems, es, offset):
    """Byte address and in-range flag of a buffer access through the fused
    passes' slice descriptor (base + (plane * plane_elems + slice *
    slice_elems) * es, range slice_elems * es, 32-bit lane offset)."""
    desc = base + (plane * plane_elems + slice_idx * slice_elems) * es
    rng = (slice_elems * es) & MASK32
    return desc + offset, offset < rng


MASK32 = 0xFFFFFFFF


@pytest.mark.parametrize("dims,es", [((1024, 1024, 1024), 4), ((1625, 1625, 1625), 2), ((2048, 2048, 300), 4),
                                     ((32768, 32768, 1), 4), ((65536, 65535, 1), 2), ((7, 5, 3), 4)])
def test_slice_descriptors_address_every_site(dims, es):
    """Planes of 4 GiB or more are addressed one z-plane (D3Q19) or one row
    (D2Q9, nz = 1) per descriptor: for sampled sites of every population
    plane (the last site included) the descriptor base, its range and the
    lane offset give the site's byte address in the (q, nz, ny, nx) state,
    with the offset inside the descriptor's range; the slice fits a 32-bit
    range (the condition under which the library accepts the fused
    schedule), while the whole plane may not."""
    nx, ny, nz = dims
    q = 9 if nz == 1 else 19
    base = 1 << 40
    plane = nx * ny * nz
    if nz == 1:  # rows
        slice_elems, nslices = nx, ny
    else:        # z-planes
        slice_elems, nslices = nx * ny, nz
    assert slice_elems * es < 2 ** 32
    rng = np.random.default_rng(nx + ny + nz)
    sites = list(rng.integers(0, plane, size=200)) + [0, plane - 1, slice_elems - 1, slice_elems, plane - slice_elems]
    for i in (0, 1, q - 1):
        for s in sites:
            s = int(s)
            sl, within = divmod(s, slice_elems)
            assert sl < nslices
            addr, ok = _slice_access(base, plane, i, sl, slice_elems, es, within * es)
            assert ok and addr == base + (i * plane + s) * es, (dims, i, s)
