"""Host-side replay of the index algebra of the in-place (AA) step kernels.

The step kernels update one state buffer in place without any
synchronisation.  That is only safe if, in every step, each thread reads and
writes the same set of (plane, site) locations and no two threads share a
location.  This test replays, with plain integers, the addressing the kernels
use (32-bit wrap-around neighbour offsets, invariant-divisor division for
the site coordinates, the flat and row tilings, the XCD tile remaps) and
checks on small boxes, where neighbours alias, that:
  - every thread's read set equals its write set;
  - the sets of different threads are disjoint and cover all q planes;
  - an even step followed by an odd step with the identity collision moves
    every population by c_i per step (Eq. LBE's streaming, periodic), and
    the parity-resolved reading of the odd state is the once-shifted state;
  - the invariant-divisor division equals integer division over the whole
    32-bit range for the divisors a box can have;
  - every XCD remap is a bijection on the workgroup indices.
It needs no GPU: it checks the design, and the GPU parity tests check the
compiled kernels against the oracle on the same boxes."""
import itertools

import numpy as np
import pytest

import oracle

MASK = 0xFFFFFFFF
C, _A, _E, _W = oracle.tables()
Q = len(C)
OPP = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, Q)]


def div_magic(d):
    """Granlund-Montgomery constants for division by d (32-bit)."""
    l = 0
    while (1 << l) < d:
        l += 1
    m = ((1 << 32) * ((1 << l) - d)) // d + 1
    return m & MASK, (1 if l > 0 else 0), (l - 1 if l > 0 else 0)


def fastdiv(n, magic):
    m, s1, s2 = magic
    t = (n * m) >> 32
    return ((t + (((n - t) & MASK) >> s1)) & MASK) >> s2


class Box:
    def __init__(self, nx, ny, nz):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        self.nxy = nx * ny
        self.wx, self.wy, self.wz = nx - 1, (ny - 1) * nx, (nz - 1) * nx * ny
        self.dx = div_magic(nx)
        self.dy = div_magic(ny)

    def steps(self, x, y, z):
        """Periodic +-1 steps along x, y, z as 32-bit wrap-around offsets."""
        xm = self.wx if x == 0 else MASK
        xp = (-self.wx) & MASK if x == self.wx else 1
        ym = self.wy if y == 0 else (-self.nx) & MASK
        yp = (-self.wy) & MASK if y * self.nx == self.wy else self.nx
        zm = self.wz if z == 0 else (-self.nxy) & MASK
        zp = (-self.wz) & MASK if z * self.nxy == self.wz else self.nxy
        return (xm, xp), (ym, yp), (zm, zp)

    def neighbour_offsets(self, site):
        """Offsets of site + c_j for every j (the flat tiling's odd step)."""
        zy = fastdiv(site, self.dx)
        x = site - zy * self.nx
        z = fastdiv(zy, self.dy)
        y = zy - z * self.ny
        (xm, xp), (ym, yp), (zm, zp) = self.steps(x, y, z)
        out = []
        for cx, cy, cz in C:
            s = site
            s += yp if cy > 0 else (ym if cy < 0 else 0)
            s += zp if cz > 0 else (zm if cz < 0 else 0)
            s += xp if cx > 0 else (xm if cx < 0 else 0)
            out.append(s & MASK)
        return out


def flat_threads(box, block, parity):
    """(reads, writes) per thread of the flat tiling: lists of (plane, site)."""
    threads = []
    G = (box.N + block - 1) // block
    for b in range(G):
        for lane in range(block):
            site = b * block + lane
            if site >= box.N:
                continue
            if parity == 0:
                reads = [(i, site) for i in range(Q)]
                writes = [(OPP[i], site) for i in range(Q)]
            else:
                o = box.neighbour_offsets(site)
                reads = [(j, o[j]) for j in range(Q)]
                writes = [(j, o[j]) for j in range(Q)]
            threads.append((site, reads, writes))
    return threads


def row_threads(box, block, parity):
    """The same for the row tiling: workgroup bl takes segment bl % segs of
    row bl // segs (row = y + ny z); lanes past the row's end stay idle."""
    segs = (box.nx + block - 1) // block
    dseg = div_magic(segs)
    threads = []
    for bl in range(box.ny * box.nz * segs):
        row = fastdiv(bl, dseg)
        for lane in range(block):
            x = (bl - row * segs) * block + lane
            if x >= box.nx:
                continue
            z = fastdiv(row, box.dy)
            y = row - z * box.ny
            r0 = row * box.nx
            site = x + r0
            _, (ym, yp), (zm, zp) = box.steps(x, y, z)
            bxm = box.wx if x == 0 else x - 1
            bxp = 0 if x == box.wx else x + 1
            if parity == 0:
                reads = [(i, (r0 + x) & MASK) for i in range(Q)]
                writes = [(OPP[i], (r0 + x) & MASK) for i in range(Q)]
            else:
                locs = []
                for j, (cx, cy, cz) in enumerate(C):
                    ro = r0
                    ro += yp if cy > 0 else (ym if cy < 0 else 0)
                    ro += zp if cz > 0 else (zm if cz < 0 else 0)
                    vx = bxp if cx > 0 else (bxm if cx < 0 else x)
                    locs.append((j, (ro + vx) & MASK))
                reads, writes = locs, locs
            threads.append((site, reads, writes))
    return threads


BOXES = [(1, 1, 1), (2, 2, 2), (3, 2, 5), (4, 3, 2), (7, 1, 1), (1, 1, 9), (5, 9, 3)]


@pytest.mark.parametrize("dims", BOXES)
@pytest.mark.parametrize("tiling", ["flat", "rows"])
@pytest.mark.parametrize("block", [4, 64])
def test_each_thread_owns_its_locations(dims, tiling, block):
    box = Box(*dims)
    make = flat_threads if tiling == "flat" else row_threads
    for parity in (0, 1):
        threads = make(box, block, parity)
        assert sorted(t[0] for t in threads) == list(range(box.N))  # every site exactly once
        seen = set()
        for site, reads, writes in threads:
            assert sorted(reads) == sorted(writes), (site, parity)
            assert len(set(reads)) == Q, (site, parity)  # no location twice within a thread
            for plane, off in reads:
                assert 0 <= off < box.N, (site, plane, off)
            assert seen.isdisjoint(reads), (site, parity)
            seen.update(reads)
        assert len(seen) == Q * box.N


def _apply(threads, state, parity):
    """One step with the identity collision, the way the kernels move data:
    every thread loads all its populations, then stores them."""
    new = state.copy()
    for site, reads, _ in threads:
        if parity == 0:
            vals = {i: state[p, o] for i, (p, o) in enumerate(reads)}  # population i of site
            for i in range(Q):
                new[OPP[i], site] = vals[i]
        else:
            # plane j at r + c_j holds population opp(j) of r; population j goes to plane j at r + c_j
            pops = {OPP[j]: state[p, o] for j, (p, o) in enumerate(reads)}
            for j, (p, o) in enumerate(reads):
                new[p, o] = pops[j]
    return new


def _resolve(box, state, parity):
    """Parity-resolved populations n_i(r) from the AA state."""
    n = np.empty_like(state)
    for site in range(box.N):
        if parity == 0:
            for i in range(Q):
                n[i, site] = state[i, site]
        else:
            o = box.neighbour_offsets(site)
            for j in range(Q):
                n[OPP[j], site] = state[j, o[j]]
    return n


def _shift(box, n, k):
    """n_i(r) -> n_i(r - k c_i): k steps of periodic push streaming."""
    out = np.empty_like(n)
    for i, (cx, cy, cz) in enumerate(C):
        g = n[i].reshape(box.nz, box.ny, box.nx)
        out[i] = np.roll(g, shift=(k * cz, k * cy, k * cx), axis=(0, 1, 2)).ravel()
    return out


@pytest.mark.parametrize("dims", BOXES)
@pytest.mark.parametrize("tilings", [("flat", "flat"), ("rows", "flat"), ("flat", "rows"), ("rows", "rows")])
def test_two_steps_stream_every_population(dims, tilings):
    box = Box(*dims)
    rng = np.random.default_rng(11)
    n0 = rng.normal(size=(Q, box.N))
    state = n0.copy()  # the even layout holds n_i(r) in plane i at r
    for parity, tiling in enumerate(tilings):
        make = flat_threads if tiling == "flat" else row_threads
        state = _apply(make(box, 64, parity), state, parity)
        np.testing.assert_array_equal(_resolve(box, state, (parity + 1) % 2), _shift(box, n0, parity + 1))


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 9, 17, 511, 512, 513, 768, 1625, 65535, 65536, 2 ** 20 + 3])
def test_invariant_division(d):
    magic = div_magic(d)
    rng = np.random.default_rng(d)
    ns = list(rng.integers(0, 2 ** 32, 4000, dtype=np.uint64)) + [0, 1, d - 1, d, d + 1, MASK, MASK - 1]
    ns += [k * d + r for k in (1, 2, 1000, (MASK // d)) for r in (0, d - 1) if k * d + r <= MASK]
    for n in ns:
        n = int(n)
        assert fastdiv(n, magic) == n // d, (d, n)


def xcd_remap(i, G, mode):
    if mode == 0:
        return i
    if mode == 1:
        q, r, x, k = G >> 3, G & 7, i & 7, i >> 3
        return x * q + (x if x < r else r) + k
    S = 8 * mode
    full = (G // S) * S
    if i >= full:
        return i
    base, r = i - i % S, i % S
    return base + (r & 7) * mode + (r >> 3)


@pytest.mark.parametrize("G", [1, 7, 8, 9, 63, 64, 65, 1000, 4099, 65536])
@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 8, 64])
def test_xcd_remap_is_a_bijection(G, mode):
    got = sorted(xcd_remap(i, G, mode) for i in range(G))
    assert got == list(range(G))
