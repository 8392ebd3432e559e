"""Tile placement of the multi-step kernels (host-side checks of the index rules the kernels
use; no GPU).

Two steps per launch with walls through the boundary nodes: in the second step a boundary node
rebuilds its populations by non-equilibrium extrapolation from its neighbours f and ff along the
inward normal (the inward diagonal at a corner), whose own pre-collision populations are pulled
from the first step's results held in LDS for the tile and a one-node halo ring.  The kernel
places the last tile of each row and column against the far wall, x0 = min(t W, nx - W),
y0 = min(t H, ny - H).  The first tests check, for every tile of many lattice shapes, that every
LDS read of that rule stays in the tile's region and lands on a node the first step computed,
and that a tile the kernel treats as interior holds no boundary node in its region.  The last
ones check the region bookkeeping of three steps per launch and that the order in which a launch
visits its tiles (row by row or in vertical strips) covers every tile once.
"""
import pytest

# two-step tiles: 64 x 8 (FP32, FP16 storage) and 32 x 8 (FP64)
TILES = [(64, 8), (32, 8)]


def _check_lattice(W, H, nx, ny, perx, pery):
    RW, RH = W + 2, H + 2
    ntx, nty = -(-nx // W), -(-ny // H)

    def boundary(X, Y):
        return (not perx and X in (0, nx - 1)) or (not pery and Y in (0, ny - 1))

    for ty in range(nty):
        for tx in range(ntx):
            x0, y0 = min(tx * W, nx - W), min(ty * H, ny - H)
            assert x0 >= 0 and y0 >= 0
            interior = x0 >= 2 and x0 + W + 1 <= nx - 1 and y0 >= 2 and y0 + H + 1 <= ny - 1
            if interior:
                for lx in range(RW):
                    for ly in range(RH):
                        X, Y = x0 - 1 + lx, y0 - 1 + ly
                        assert 0 <= X < nx and 0 <= Y < ny and not boundary(X, Y)
                continue

            def computed(lx, ly):
                # the first step skips region nodes beyond a wall; across a periodic side it
                # computes the wrapped node
                X, Y = x0 - 1 + lx, y0 - 1 + ly
                return (perx or 0 <= X < nx) and (pery or 0 <= Y < ny)

            for t in range(W * H):
                x, y = x0 + t % W, y0 + t // W
                assert x < nx and y < ny
                bx = not perx and x in (0, nx - 1)
                by = not pery and y in (0, ny - 1)
                if not (bx or by):
                    continue
                dx = (1 if x == 0 else -1) if bx else 0
                dy = (1 if y == 0 else -1) if by else 0
                for k in (1, 2):                       # f and ff
                    px, py = x + k * dx, y + k * dy
                    assert 0 <= px < nx and 0 <= py < ny
                    cx, cy = px - x0 + 1, py - y0 + 1
                    for ex in (-1, 0, 1):              # the node and its eight upstream nodes
                        for ey in (-1, 0, 1):
                            lx, ly = cx + ex, cy + ey
                            assert 0 <= lx < RW and 0 <= ly < RH, (W, H, nx, ny, x, y, k)
                            assert computed(lx, ly), (W, H, nx, ny, perx, pery, x, y, lx, ly)


@pytest.mark.parametrize("W,H", TILES)
def test_boundary_rule_reads_stay_in_the_tile_region(W, H):
    sizes_x = list(range(W, W + 9)) + list(range(2 * W - 3, 2 * W + 4)) + [3 * W + 1, 100, 129, 200]
    sizes_y = list(range(H, H + 10)) + [2 * H - 1, 2 * H + 1, 37, 70, 129, 257]
    n = 0
    for nx in sizes_x:
        for ny in sizes_y:
            for perx, pery in ((False, False), (True, False), (False, True)):
                _check_lattice(W, H, nx, ny, perx, pery)
                n += 1
    assert n == len(sizes_x) * len(sizes_y) * 3


def test_a_misplaced_last_tile_is_caught():
    """The same check with the last tile left ragged (x0 = t W) fails on a lattice whose last
    column of tiles is narrower than three nodes."""
    W, H, nx, ny = 64, 8, 66, 16
    ragged_x0 = (nx // W) * W                      # 64: the tile holds columns 64, 65 only
    px = (nx - 1) - 2                              # ff of the right-wall node
    assert px - ragged_x0 + 1 - 1 < 0              # its upstream column falls outside the region
    _check_lattice(W, H, nx, ny, False, False)     # the placement the kernel uses passes


# ---------------------------------------------------------------- three steps per launch
# The three-step kernel keeps a two-node halo: step one computes the (W + 4) x (H + 4) region,
# step two the inner (W + 2) x (H + 2) region in place, step three the tile.  Each region node
# belongs to one thread: its tile node, an inner-ring node (threads [0, N1)) or an outer-ring
# node (threads [N1, N1 + N2)).  The check below walks, for every tile, every node the third
# step stores, the region nodes its pulls read in step two and theirs in step one, and checks
# that each was computed by the previous step and holds a node of the domain (across a periodic
# side: the wrapped one).
def _check_three_step(W, H, nx, ny, perx, pery):
    RW, RH = W + 4, H + 4
    N1 = 2 * (W + 2) + 2 * H
    N2 = 2 * RW + 2 * (H + 2)
    assert N1 + N2 <= W * H
    own = {(t % W + 2, t // W + 2) for t in range(W * H)}
    r1, r2 = set(), set()
    for t in range(N1 + N2):
        if t < N1:
            if t < 2 * (W + 2):
                rx, ry = 1 + t % (W + 2), (1 if t < W + 2 else RH - 2)
            else:
                q = t - 2 * (W + 2)
                rx, ry = (1 if q < H else RW - 2), 2 + q % H
            assert (rx, ry) not in r1
            r1.add((rx, ry))
        else:
            k = t - N1
            if k < 2 * RW:
                rx, ry = k % RW, (0 if k < RW else RH - 1)
            else:
                q = k - 2 * RW
                rx, ry = (0 if q < H + 2 else RW - 1), 1 + q % (H + 2)
            assert (rx, ry) not in r2
            r2.add((rx, ry))
    assert not (own & r1) and not (own & r2) and not (r1 & r2)
    assert own | r1 | r2 == {(x, y) for x in range(RW) for y in range(RH)}
    inner = own | r1
    assert inner == {(x, y) for x in range(1, RW - 1) for y in range(1, RH - 1)}
    ntx, nty = -(-nx // W), -(-ny // H)
    for ty_ in range(nty):
        for tx_ in range(ntx):
            x0, y0 = tx_ * W, ty_ * H
            interior = x0 >= 3 and x0 + W + 2 <= nx - 1 and y0 >= 3 and y0 + H + 2 <= ny - 1
            def locate(lx, ly):
                X, Y = x0 - 2 + lx, y0 - 2 + ly
                if not (0 <= X < nx):
                    if not perx:
                        return None
                    X = X + nx if X < 0 else X - nx
                if not (0 <= Y < ny):
                    if not pery:
                        return None
                    Y = Y + ny if Y < 0 else Y - ny
                return X, Y
            if interior:
                for lx in range(RW):
                    for ly in range(RH):
                        X, Y = x0 - 2 + lx, y0 - 2 + ly
                        assert 1 <= X <= nx - 2 and 1 <= Y <= ny - 2
            def valid(p):
                q = locate(*p)
                return q is not None and 0 <= q[0] < nx and 0 <= q[1] < ny
            step1 = {p for p in own | r1 | r2 if locate(*p) is not None}
            step2 = {p for p in inner if locate(*p) is not None}
            def sources(p):
                X, Y = locate(*p)
                out = []
                for ex in (-1, 0, 1):
                    for ey in (-1, 0, 1):
                        okx = (ex == 0) or perx or (0 <= X - ex < nx)
                        oky = (ey == 0) or pery or (0 <= Y - ey < ny)
                        if okx and oky:
                            out.append((p[0] - ex, p[1] - ey))
                return out
            for p in own:
                X, Y = x0 + p[0] - 2, y0 + p[1] - 2
                if X < nx and Y < ny:
                    for q in sources(p):                 # step three reads step two at q
                        assert q in step2 and valid(q), (p, q)
                        # the wrapped node at q pulls the same neighbours as the real one
                        for r_ in sources(q):            # step two at q reads step one at r_
                            assert r_ in step1 and valid(r_), (p, q, r_)


@pytest.mark.parametrize("W,H", TILES + [(64, 12)])
def test_three_step_rings_cover_the_region_and_feed_every_stored_node(W, H):
    for nx in (3, 5, 65, 70, 129):
        for ny in (3, 5, 9, 37):
            for perx, pery in ((False, False), (True, False), (False, True), (True, True)):
                _check_three_step(W, H, nx, ny, perx, pery)


def _tile_of(b, ntx, nty, sw):
    """The kernels' tile order: row by row (sw = 0, or sw >= ntx), or vertical strips of sw
    tiles, the last one narrower, each walked row by row."""
    if sw <= 0 or sw >= ntx:
        return b % ntx, b // ntx
    st = sw * nty
    s, rem = divmod(b, st)
    ws = min(sw, ntx - s * sw)
    return s * sw + rem % ws, rem // ws


@pytest.mark.parametrize("sw", [0, 1, 2, 3, 4, 5, 8, 16, 64])
def test_tile_order_is_a_permutation(sw):
    """Every tile of the launch grid is visited once, for every strip width and grid shape."""
    for ntx in list(range(1, 40)) + [64, 128, 234]:
        for nty in (1, 2, 5, 8, 33, 256):
            seen = {_tile_of(b, ntx, nty, sw) for b in range(ntx * nty)}
            assert len(seen) == ntx * nty, (ntx, nty)
            assert all(0 <= x < ntx and 0 <= y < nty for x, y in seen), (ntx, nty)
    # within a full strip, consecutive tiles run along a row of the strip, then down
    assert [_tile_of(b, 10, 3, 4) for b in range(6)] == [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (1, 1)]
    assert _tile_of(24, 10, 3, 4) == (8, 0) and _tile_of(25, 10, 3, 4) == (9, 0) and _tile_of(26, 10, 3, 4) == (8, 1)
