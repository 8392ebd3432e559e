"""Autotune cache bookkeeping (no GPU: a stand-in solver reports timings)."""
from paper_1708_07525_amd import autotune


class FakeSolver:
    def __init__(self, nx, ny, precision="fp32"):
        self.nx, self.ny, self.precision = nx, ny, precision
        self.tile = (256, 1)
        self.policy = -1
        self.timed = 0

    def autotune(self, steps):
        self.timed += 1
        self.tile = (128, 2)
        self.policy = 1
        return self.tile, 0.25

    def set_tile(self, tx, ty):
        self.tile = (tx, ty)

    def set_cache_policy(self, p):
        self.policy = p

    def get_cache_policy(self):
        return self.policy

    def set_steps_per_launch(self, n):
        self.spl = n

    def get_steps_per_launch(self):
        return getattr(self, "spl", 2)

    def set_strip_width(self, n):
        self.strip = n

    def get_strip_width(self):
        return getattr(self, "strip", 4)

    def set_tile_rows(self, n):
        self.rows = n

    def get_tile_rows(self):
        return getattr(self, "rows", 12)


def test_size_class_and_key():
    assert [autotune.size_class(n) for n in (1, 3, 64, 65, 2048)] == [1, 4, 64, 128, 2048]
    g = f"g{autotune.KERNEL_GENERATION}"
    assert autotune.key("MI355X", "fp32", 100, 200, True) == g + "|MI355X|fp32|128x256|field"
    assert autotune.key("MI355X", "fp32", 100, 200, True, node_walls=True) == g + "|MI355X|fp32|128x256|field|node-walls"


def test_tune_times_once_per_class(tmp_path):
    path = str(tmp_path / "cache.json")
    a = FakeSolver(100, 100)
    assert autotune.tune(a, "gpu", False, path=path) == ((128, 2), 0.25)
    assert a.timed == 1
    b = FakeSolver(120, 90)          # same class: 128x128, uniform, fp32
    b.tile = (64, 8)
    assert autotune.tune(b, "gpu", False, path=path) == ((128, 2), None)
    assert b.timed == 0 and b.tile == (128, 2) and b.policy == 1 and b.strip == 4 and b.rows == 12
    c = FakeSolver(120, 90, "fp16s")  # other precision: timed again
    autotune.tune(c, "gpu", False, path=path)
    assert c.timed == 1
    assert len(autotune.load(path)) == 2


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "cache.json"
    path.write_text("{not json")
    s = FakeSolver(64, 64)
    autotune.tune(s, "gpu", True, path=str(path))
    assert s.timed == 1 and autotune.load(str(path))


def test_wall_families_are_tuned_apart(tmp_path):
    path = str(tmp_path / "cache.json")
    a = FakeSolver(100, 100)
    autotune.tune(a, "gpu", False, path=path)
    b = FakeSolver(100, 100)
    autotune.tune(b, "gpu", False, path=path, node_walls=True)
    assert a.timed == 1 and b.timed == 1 and len(autotune.load(path)) == 2
