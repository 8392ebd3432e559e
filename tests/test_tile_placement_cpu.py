"""Tile placement of the two-step kernel with walls through the boundary nodes (host-side
check of the index rules the kernel uses; no GPU).

In the second step a boundary node rebuilds its populations by non-equilibrium extrapolation
from its neighbours f and ff along the inward normal (the inward diagonal at a corner), whose
own pre-collision populations are pulled from the first step's results held in LDS for the
tile and a one-node halo ring.  The kernel places the last tile of each row and column against
the far wall, x0 = min(t W, nx - W), y0 = min(t H, ny - H).  These tests check, for every tile
of many lattice shapes, that every LDS read of that rule stays in the tile's region and lands
on a node the first step computed, and that a tile the kernel treats as interior holds no
boundary node in its region.
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
